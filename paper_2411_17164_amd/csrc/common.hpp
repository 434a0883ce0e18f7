// Device building blocks shared by the xmgn kernels (gfx950, wave64).
//
// A workgroup is 256 threads = 4 waves.  A row tile of MT rows is staged in
// LDS; each wave owns a quarter of the output columns of every GEMM and all
// MT rows.  Matrix products use the 16x16 MFMA instructions:
//   BF16 : v_mfma_f32_16x16x32_bf16 (8 bf16 per lane per operand)
//   FP32 : v_mfma_f32_16x16x4_f32   (1 float per lane; 4 issued per 16 bytes)
// Each lane loads 16 contiguous bytes of an A row and of a B column (B is
// given as W[n][k], i.e. k contiguous).  Lane group g = lane / 16 holds the
// k slice [g*E, g*E + E) of every 4*E-wide k chunk, identically for A and B,
// so the products sum over exactly the chunk's k range.
// Accumulator layout (16x16 block, 4 floats per lane):
//   value r of lane l is C[row = 4*(l/16) + r][col = l % 16].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xmgn {

typedef __bf16 bf16;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int NTHR = 256;
constexpr int NWAVE = 4;

template <typename T>
struct TT;
template <>
struct TT<bf16> {
  static constexpr int E = 8;  // elements per 16-byte fragment
  using V = bf16x8;
};
template <>
struct TT<float> {
  static constexpr int E = 4;
  using V = f32x4;
};

__device__ __forceinline__ f32x4 mma(const bf16x8& a, const bf16x8& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma(const f32x4& a, const f32x4& b, f32x4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], c, 0, 0, 0);
  return c;
}

__device__ __forceinline__ float to_f(float x) { return x; }
__device__ __forceinline__ float to_f(bf16 x) { return (float)x; }
template <typename T>
__device__ __forceinline__ T from_f(float x);
template <>
__device__ __forceinline__ float from_f<float>(float x) { return x; }
template <>
__device__ __forceinline__ bf16 from_f<bf16>(float x) { return (bf16)x; }

// Workgroup barrier for LDS traffic only.  The fences are restricted to the
// LDS address space, so a wave waits for its own LDS accesses (lgkmcnt)
// before the barrier but not for its global loads and stores (vmcnt): loads
// issued ahead of their use (the next tile's indices, weight fragments) stay
// in flight across it, and stores drain behind the following work.  No
// kernel that uses it reads global memory written by another thread of the
// same launch.
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// Activation and its derivative (0 = ReLU, 1 = SiLU).
template <int ACT>
__device__ __forceinline__ float act_f(float a) {
  if constexpr (ACT == 0) {
    return a > 0.f ? a : 0.f;
  } else {
    return a / (1.f + __expf(-a));
  }
}
template <int ACT>
__device__ __forceinline__ float act_d(float a) {
  if constexpr (ACT == 0) {
    return a > 0.f ? 1.f : 0.f;
  } else {
    float s = 1.f / (1.f + __expf(-a));
    return s * (1.f + a * (1.f - s));
  }
}

// The B operand B[k][n] = W[n][k] of a wave's product, for its output
// columns [n0, n0 + 16 NB) and k in [0, K), W in global memory (row stride
// ldw).  When the whole operand fits in 96 registers (BF16 at H = 128),
// load() brings every fragment in one batch, so the weights cost one round
// trip per product.  Otherwise (FP32, H = 256) the fragments are loaded
// inside the product's k loop instead.
template <typename T, int NB, int K>
struct WFrag {
  using V = typename TT<T>::V;
  static constexpr int E = TT<T>::E, KC = 4 * E;
  static constexpr bool PRE = sizeof(T) == 2 && (K / KC) * NB * 4 <= 96;
  static_assert(K % KC == 0, "K must be a multiple of the MFMA k chunk");
  V b[PRE ? K / KC : 1][NB];
  const T* wrow[NB];
  __device__ __forceinline__ void load(const T* __restrict__ W, int ldw, int n0) {
    const int l = lane_id(), li = l & 15, lg = l >> 4;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) wrow[nb] = W + (size_t)(n0 + nb * 16 + li) * ldw + lg * E;
    if constexpr (PRE) {
#pragma unroll
      for (int kk = 0; kk < K / KC; ++kk)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) b[kk][nb] = *(const V*)(wrow[nb] + kk * KC);
    }
  }
};

// acc[MB][NB] += A * B over k in [0, K):  A rows [0, 16 MB) from LDS (row
// stride LDA elements), B from a loaded WFrag.
template <typename T, int MB, int NB, int K, int LDA>
__device__ __forceinline__ void wave_gemm(f32x4 (&acc)[MB][NB], const T* A, const WFrag<T, NB, K>& f) {
  using V = typename TT<T>::V;
  constexpr int KC = WFrag<T, NB, K>::KC, E = WFrag<T, NB, K>::E;
  const int l = lane_id(), li = l & 15, lg = l >> 4;
  const T* arow = A + li * LDA + lg * E;
  if constexpr (WFrag<T, NB, K>::PRE) {
    // A fragments (LDS) are read at most two k steps ahead of their MFMAs
    // (one for tall tiles): hoisting all of them would cost K / KC x MB x 4
    // registers
    constexpr int G = MB >= 8 ? 1 : 2;
#pragma unroll
    for (int kk = 0; kk < K / KC; kk += G) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k2 = kk; k2 < kk + G && k2 < K / KC; ++k2)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          V a = *(const V*)(arow + mb * 16 * LDA + k2 * KC);
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mma(a, f.b[k2][nb], acc[mb][nb]);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
  } else {
#pragma unroll 4
    for (int k = 0; k < K; k += KC) {
      V b[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) b[nb] = *(const V*)(f.wrow[nb] + k);
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        V a = *(const V*)(arow + mb * 16 * LDA + k);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mma(a, b[nb], acc[mb][nb]);
      }
    }
  }
}

// acc[MB][NB] += A * W^T with the weight fragments loaded on the spot.
template <typename T, int MB, int NB, int K, int LDA>
__device__ __forceinline__ void wave_gemm(f32x4 (&acc)[MB][NB], const T* A,
                                          const T* __restrict__ W, int ldw, int n0) {
  WFrag<T, NB, K> f;
  f.load(W, ldw, n0);
  wave_gemm<T, MB, NB, K, LDA>(acc, A, f);
}

// The same product with A's rows taken through an indirection: this lane's
// row of 16-row block mb starts at A + roff[mb] (an LDS offset in elements,
// the lane's own row, lane % 16, of that block).
template <typename T, int MB, int NB, int K>
__device__ __forceinline__ void wave_gemm_rows(f32x4 (&acc)[MB][NB], const T* A, const int (&roff)[MB],
                                               const WFrag<T, NB, K>& f) {
  using V = typename TT<T>::V;
  constexpr int KC = WFrag<T, NB, K>::KC, E = WFrag<T, NB, K>::E;
  const int lg = lane_id() >> 4;
  if constexpr (WFrag<T, NB, K>::PRE) {
#pragma unroll
    for (int kk = 0; kk < K / KC; kk += 2) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k2 = kk; k2 < kk + 2 && k2 < K / KC; ++k2)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          V a = *(const V*)(A + roff[mb] + lg * E + k2 * KC);
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mma(a, f.b[k2][nb], acc[mb][nb]);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
  } else {
#pragma unroll 4
    for (int k = 0; k < K; k += KC) {
      V b[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) b[nb] = *(const V*)(f.wrow[nb] + k);
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        V a = *(const V*)(A + roff[mb] + lg * E + k);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mma(a, b[nb], acc[mb][nb]);
      }
    }
  }
}

// Transposing LDS read (ds_read_b64_tr_b16, gfx950).  In each group of 16
// lanes, lane L reads four 16-bit values at its own address, and lane 4a + b
// receives value b of lanes a, a + 4, a + 8 and a + 12.  So if lane L points
// at row r0 + L / 4, columns c0 + 4 (L % 4) .. + 3 of a row-major tile, lane
// j of the group gets column c0 + j of rows r0 .. r0 + 3: a k-major MFMA
// operand read from an n-major tile.
typedef __bf16 bf16x4_lds __attribute__((__vector_size__(4 * sizeof(__bf16))));
__device__ __forceinline__ bf16x4_lds lds_read_tr4(const bf16* p) {
  return __builtin_amdgcn_ds_read_tr16_b64_v4bf16((__attribute__((address_space(3))) bf16x4_lds*)(p));
}

// MFMA B fragment B[k][n] = M[k][n] (M row-major in LDS, row stride LD) for
// k in [k0 + 8 g, k0 + 8 g + 8) of lane group g and n = c0 + lane % 16.
// rows_hi is the row distance of the second half of the 8 k values (4 for
// consecutive k; any other value gives a permuted k order that the A operand
// must share).
__device__ __forceinline__ bf16x8 lds_bfrag_tr(const bf16* M, int LD, int r0, int c0, int rows_hi) {
  const int l = lane_id(), L = l & 15;
  const bf16* p = M + (size_t)(r0 + (L >> 2)) * LD + c0 + 4 * (L & 3);
  const bf16x4_lds lo = lds_read_tr4(p), hi = lds_read_tr4(p + (size_t)rows_hi * LD);
  return bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

// acc[MB][NB] += A * B over k in [0, K) for BF16, A rows from LDS (stride
// LDA), B fragments from bfrag(k, nb) (LDS-resident weights).
template <int MB, int NB, int K, int LDA, typename BFrag>
__device__ __forceinline__ void wave_gemm_lds(f32x4 (&acc)[MB][NB], const bf16* A, BFrag bfrag) {
  const int l = lane_id(), li = l & 15, lg = l >> 4;
  const bf16* arow = A + li * LDA + lg * 8;
#pragma unroll
  for (int k = 0; k < K; k += 32) {
    bf16x8 b[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) b[nb] = bfrag(k, nb);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const bf16x8 a = *(const bf16x8*)(arow + mb * 16 * LDA + k);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mma(a, b[nb], acc[mb][nb]);
    }
  }
}

template <int MB, int NB>
__device__ __forceinline__ void zero_acc(f32x4 (&acc)[MB][NB]) {
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// Row / column of value r of block (mb, nb) for this lane.
__device__ __forceinline__ int acc_row(int mb, int r) { return mb * 16 + (lane_id() >> 4) * 4 + r; }
__device__ __forceinline__ int acc_col(int n0, int nb) { return n0 + nb * 16 + (lane_id() & 15); }

// Sum over the 16 lanes of a DPP row (same rows, 16 columns), with DPP lane
// moves (no LDS traffic): pairs (quad_perm 1,0,3,2), quads (2,3,0,1),
// halves (row_half_mirror) and the two halves of the row (row_mirror).  Each
// step adds a lane to its partner, so every lane ends with the same sum.
template <int CTRL>
__device__ __forceinline__ float dpp_add(float s) {
  const int v = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, s), CTRL, 0xF, 0xF, false);
  return s + __builtin_bit_cast(float, v);
}
__device__ __forceinline__ float sum16(float s) {
  s = dpp_add<0xB1>(s);   // quad_perm [1,0,3,2]
  s = dpp_add<0x4E>(s);   // quad_perm [2,3,0,1]
  s = dpp_add<0x141>(s);  // row_half_mirror
  s = dpp_add<0x140>(s);  // row_mirror
  return s;
}
// Sum over the 4 lane groups (same column, 4 x 4 rows).
__device__ __forceinline__ float sum_groups(float s) {
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  return s;
}

// Full-row sums of x over all columns of all NW waves.  red: LDS float
// [NW][MT].  Returns out[mb][r] = sum over the row acc_row(mb, r), the wave
// partials added in wave order.  Contains two barriers.
template <int MB, int NB, int MT, int NW = NWAVE>
__device__ __forceinline__ void row_sum(const f32x4 (&x)[MB][NB], float* red, float (&out)[MB][4]) {
  const int w = wave_id(), l = lane_id();
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float s = 0.f;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) s += x[mb][nb][r];
      s = sum16(s);
      if ((l & 15) == 0) red[w * MT + acc_row(mb, r)] = s;
    }
  lds_sync();
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = acc_row(mb, r);
      float t = 0.f;
#pragma unroll
      for (int k = 0; k < NW; k += 2) t += red[k * MT + row] + red[(k + 1) * MT + row];
      out[mb][r] = t;
    }
  lds_sync();
}

// Two row sums (of x and of y) exchanged across the NW waves in one barrier
// round.  red: LDS float [2][NW][MT].
template <int MB, int NB, int MT, int NW = NWAVE>
__device__ __forceinline__ void row_sum2(const f32x4 (&x)[MB][NB], const f32x4 (&y)[MB][NB], float* red,
                                         float (&ox)[MB][4], float (&oy)[MB][4]) {
  const int w = wave_id(), l = lane_id();
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float a = 0.f, c = 0.f;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        a += x[mb][nb][r];
        c += y[mb][nb][r];
      }
      a = sum16(a);
      c = sum16(c);
      if ((l & 15) == 0) {
        red[w * MT + acc_row(mb, r)] = a;
        red[(NW + w) * MT + acc_row(mb, r)] = c;
      }
    }
  lds_sync();
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = acc_row(mb, r);
      float a = 0.f, c = 0.f;
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        a += red[k * MT + row];
        c += red[(NW + k) * MT + row];
      }
      ox[mb][r] = a;
      oy[mb][r] = c;
    }
  lds_sync();
}

// LayerNorm of the rows of u (in place -> xhat), returning inv std per row.
// Statistics in FP32.  Each wave takes the mean and the sum of squared
// deviations (M2) over its own H / NW columns; the waves' (mean, M2) pairs
// are merged in one barrier round with the pairwise-variance formula
// M2 = sum_w [M2_w + n_w (mean_w - mean)^2].  red: LDS float [2][NW][MT].
template <int MB, int NB, int MT, int H, int NW = NWAVE>
__device__ __forceinline__ void ln_normalize(f32x4 (&u)[MB][NB], float* red, float eps,
                                             float (&inv)[MB][4]) {
  constexpr float CPW = (float)(H / NW);
  const int w = wave_id(), l = lane_id();
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float a = 0.f;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) a += u[mb][nb][r];
      const float mw = sum16(a) * (1.f / CPW);
      float q = 0.f;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float d = u[mb][nb][r] - mw;
        q += d * d;
      }
      q = sum16(q);
      if ((l & 15) == 0) {
        red[w * MT + acc_row(mb, r)] = mw;
        red[(NW + w) * MT + acc_row(mb, r)] = q;
      }
    }
  lds_sync();
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = acc_row(mb, r);
      float mean = 0.f;
#pragma unroll
      for (int k = 0; k < NW; ++k) mean += red[k * MT + row];
      mean *= 1.f / NW;
      float m2 = 0.f;
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const float dm = red[k * MT + row] - mean;
        m2 += red[(NW + k) * MT + row] + CPW * dm * dm;
      }
      inv[mb][r] = rsqrtf(m2 * (1.f / H) + eps);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) u[mb][nb][r] = (u[mb][nb][r] - mean) * inv[mb][r];
    }
  lds_sync();
}

// Column sums of x over all rows held by the wave, accumulated into acc[nb]
// (every lane of a column ends with the same total).  The per-workgroup
// running sums over many tiles are FP64: they add up long, cancelling
// series of tile sums (bias and LayerNorm gradients).
template <int MB, int NB>
__device__ __forceinline__ void col_accumulate(const f32x4 (&x)[MB][NB], double (&acc)[NB]) {
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    float s = 0.f;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) s += (x[mb][nb][0] + x[mb][nb][1]) + (x[mb][nb][2] + x[mb][nb][3]);
    acc[nb] += (double)sum_groups(s);
  }
}

// Store the accumulator (as T) into an LDS tile with row stride LD.
template <typename T, int MB, int NB, int LD>
__device__ __forceinline__ void acc_to_lds(const f32x4 (&x)[MB][NB], T* dst, int n0) {
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[acc_row(mb, r) * LD + acc_col(n0, nb)] = from_f<T>(x[mb][nb][r]);
}

// Copy `rows` rows of `width` elements from an LDS tile (stride LD) to global
// rows dst + row_index(i) * ld_dst, 16 bytes per thread-step.
template <typename T, int LD, typename RowFn>
__device__ __forceinline__ void lds_rows_to_global(const T* src, int rows, int width, T* dst,
                                                   size_t ld_dst, RowFn row_index) {
  constexpr int E = 16 / sizeof(T);
  const int cpr = width / E;
  for (int c = threadIdx.x; c < rows * cpr; c += blockDim.x) {
    const int i = c / cpr, q = c - i * cpr;
    *(uint4*)(dst + (size_t)row_index(i) * ld_dst + q * E) = *(const uint4*)(src + i * LD + q * E);
  }
}

// Copy rows of W elements from global into an LDS tile (16-byte steps),
// zero-filling rows >= rows up to MT; a workgroup of NTHR threads, all loads
// issued before the first LDS store.
template <typename T, int LD, int MT, int W, typename SrcFn>
__device__ __forceinline__ void global_rows_to_lds(T* dst, int rows, int col0, SrcFn src_row) {
  constexpr int E = 16 / sizeof(T), CPR = W / E, TOT = MT * CPR, IT = (TOT + NTHR - 1) / NTHR;
  uint4 v[IT];
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int c = (int)threadIdx.x + k * NTHR, i = c / CPR, q = c - i * CPR;
    v[k] = uint4{0u, 0u, 0u, 0u};
    if (c < TOT && i < rows) v[k] = *(const uint4*)(src_row(i) + q * E);
  }
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int c = (int)threadIdx.x + k * NTHR, i = c / CPR, q = c - i * CPR;
    if (c < TOT) *(uint4*)(dst + i * LD + col0 + q * E) = v[k];
  }
}

// Gather a tile of MT rows x NP parts of H elements (part p of row i from
// src(p, i)) into LDS at columns p H, zero-filling rows >= rows.  The trip
// count is a compile-time constant, so every load of the tile is issued
// before the first one is waited on (one memory round trip per tile).
// hook(p, i, q, v) sees each 16-byte chunk q of part p of row i after it is
// stored.
template <typename T, int LD, int MT, int NP, int H, int NTHR, typename SrcFn, typename Hook>
__device__ __forceinline__ void gather_tile(T* dst, int rows, SrcFn src, Hook hook) {
  constexpr int E = 16 / sizeof(T), CPR = H / E, TOT = MT * NP * CPR;
  static_assert(TOT % NTHR == 0, "whole steps of the workgroup");
  constexpr int IT = TOT / NTHR;
  uint4 v[IT];
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int c = (int)threadIdx.x + k * NTHR;
    const int p = c / (MT * CPR), rem = c - p * (MT * CPR), i = rem / CPR, q = rem - i * CPR;
    v[k] = uint4{0u, 0u, 0u, 0u};
    if (i < rows) v[k] = *(const uint4*)(src(p, i) + q * E);
  }
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int c = (int)threadIdx.x + k * NTHR;
    const int p = c / (MT * CPR), rem = c - p * (MT * CPR), i = rem / CPR, q = rem - i * CPR;
    *(uint4*)(dst + i * LD + p * H + q * E) = v[k];
    hook(p, i, q, v[k]);
  }
}

// FP32 tile of MT rows x H: row i, float4 q = a(i, q) (+ b(i, q) when
// with_b), zero for rows >= rows, one batch of loads; the result goes to
// LDS (row stride LD) through put(i, q, value).
template <int MT, int H, int NTHR, typename AFn, typename BFn, typename PutFn>
__device__ __forceinline__ void f32_tile(int rows, bool with_b, AFn a, BFn b, PutFn put) {
  constexpr int CPR = H / 4, TOT = MT * CPR;
  static_assert(TOT % NTHR == 0, "whole steps of the workgroup");
  constexpr int IT = TOT / NTHR;
  float4 va[IT], vb[IT];
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int c = (int)threadIdx.x + k * NTHR, i = c / CPR, q = c - i * CPR;
    va[k] = float4{0.f, 0.f, 0.f, 0.f};
    vb[k] = float4{0.f, 0.f, 0.f, 0.f};
    if (i < rows) {
      va[k] = a(i, q);
      if (with_b) vb[k] = b(i, q);
    }
  }
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int c = (int)threadIdx.x + k * NTHR, i = c / CPR, q = c - i * CPR;
    float4 v = va[k];
    v.x += vb[k].x;
    v.y += vb[k].y;
    v.z += vb[k].z;
    v.w += vb[k].w;
    put(i, q, v);
  }
}

// The [h ; m] rows of a node tile (h in T, m in FP32) held in registers
// between their loads and their stores into an LDS tile of row stride LD
// (h at columns [0, H), m converted to T at [H, 2H), zero rows from `rows`
// on), so that a persistent node kernel can issue the next tile's loads
// while it computes the current one.  Same thread-to-chunk mapping as
// global_rows_to_lds and global_f32_rows_to_lds.
template <typename T, int H, int MT, int LD>
struct NodeRowsPre {
  static constexpr int EH = 16 / sizeof(T), CPH = H / EH, CPF = H / 4;
  static constexpr int IH = MT * CPH / NTHR, IF = MT * CPF / NTHR;
  static_assert(MT * CPH % NTHR == 0 && MT * CPF % NTHR == 0, "whole steps of the workgroup");
  uint4 vh[IH];
  float4 vm[IF];
  __device__ __forceinline__ void load(const T* __restrict__ h, const float* __restrict__ m, int row0, int rows) {
#pragma unroll
    for (int k = 0; k < IH; ++k) {
      const int c = (int)threadIdx.x + k * NTHR, i = c / CPH, q = c - i * CPH;
      vh[k] = uint4{0u, 0u, 0u, 0u};
      if (i < rows) vh[k] = *(const uint4*)(h + (size_t)(row0 + i) * H + q * EH);
    }
#pragma unroll
    for (int k = 0; k < IF; ++k) {
      const int c = (int)threadIdx.x + k * NTHR, i = c / CPF, q = c - i * CPF;
      vm[k] = float4{0.f, 0.f, 0.f, 0.f};
      if (i < rows) vm[k] = *(const float4*)(m + (size_t)(row0 + i) * H + 4 * q);
    }
  }
  __device__ __forceinline__ void store(T* xs) const {
#pragma unroll
    for (int k = 0; k < IH; ++k) {
      const int c = (int)threadIdx.x + k * NTHR, i = c / CPH, q = c - i * CPH;
      *(uint4*)(xs + i * LD + q * EH) = vh[k];
    }
#pragma unroll
    for (int k = 0; k < IF; ++k) {
      const int c = (int)threadIdx.x + k * NTHR, i = c / CPF, q = c - i * CPF;
      T* d = xs + i * LD + H + 4 * q;
      d[0] = from_f<T>(vm[k].x);
      d[1] = from_f<T>(vm[k].y);
      d[2] = from_f<T>(vm[k].z);
      d[3] = from_f<T>(vm[k].w);
    }
  }
};

// FP32 global rows of W floats converted into a T tile in LDS, zero-filling
// rows >= rows up to MT; NTHR threads, all loads issued before the stores.
template <typename T, int LD, int MT, int W, typename SrcFn>
__device__ __forceinline__ void global_f32_rows_to_lds(T* dst, int rows, int col0, SrcFn src_row) {
  constexpr int CPR = W / 4, TOT = MT * CPR, IT = (TOT + NTHR - 1) / NTHR;
  float4 v[IT];
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int c = (int)threadIdx.x + k * NTHR, i = c / CPR, q = c - i * CPR;
    v[k] = float4{0.f, 0.f, 0.f, 0.f};
    if (c < TOT && i < rows) v[k] = *(const float4*)(src_row(i) + q * 4);
  }
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int c = (int)threadIdx.x + k * NTHR, i = c / CPR, q = c - i * CPR;
    if (c < TOT) {
      T* d = dst + i * LD + col0 + q * 4;
      d[0] = from_f<T>(v[k].x);
      d[1] = from_f<T>(v[k].y);
      d[2] = from_f<T>(v[k].z);
      d[3] = from_f<T>(v[k].w);
    }
  }
}

// Waves per SIMD that the LDS footprint of a workgroup of NW waves allows
// (160 KiB of LDS per CU, 4 SIMDs), as a register budget for the compiler:
// it may then use 512 / waves registers per lane and no more.
__host__ __device__ constexpr int waves_per_simd(size_t lds_bytes, int nw) {
  const int wg = (int)((160u * 1024u) / (lds_bytes ? lds_bytes : 1));
  const int w = wg * nw / 4;
  return w < 1 ? 1 : (w > 2 ? 2 : w);
}

// Bounds of one edge tile: receivers [r0, r1), edges [e0, e1).  The plan
// stores (receiver, edge) pairs per tile boundary, so the four bounds are
// two independent loads.
struct EdgeTileBounds {
  int r0, r1, e0, e1;
  template <typename BV>
  __device__ __forceinline__ void load(const BV& b, int t) {
    const int2 lo = *(const int2*)(b.etiles + 2 * t);
    const int2 hi = *(const int2*)(b.etiles + 2 * t + 2);
    r0 = lo.x;
    e0 = lo.y;
    r1 = hi.x;
    e1 = hi.y;
  }
};

// Indices of one edge tile: its receiver range [r0, r1), its edge range
// [e0, e0 + ne), and this thread's edge (receiver rv, sender cv; threads
// below ne).
struct EdgeTileIdx {
  int r0, r1, e0, ne, rv, cv;
  template <typename BV>
  __device__ __forceinline__ void load(const BV& b, const EdgeTileBounds& bd) {
    r0 = bd.r0;
    r1 = bd.r1;
    e0 = bd.e0;
    ne = bd.e1 - bd.e0;
    rv = 0;
    cv = 0;
    if ((int)threadIdx.x < ne) {
      rv = b.recv[e0 + threadIdx.x];
      cv = b.col[e0 + threadIdx.x];
    }
  }
  // bounds and indices of tile t, one dependent step after the other
  template <typename BV>
  __device__ __forceinline__ void load(const BV& b, int t) {
    EdgeTileBounds bd;
    bd.load(b, t);
    load(b, bd);
  }
};

// Index pipeline of a persistent edge kernel: while a workgroup works on
// tile t, the per-thread indices of its next tile and the bounds of the tile
// after that are in flight, so neither link of the dependent chain
// (bounds -> indices) waits on the critical path of a tile.
struct EdgeTilePipe {
  EdgeTileBounds nb;  // bounds of the tile after the next
  EdgeTileIdx nx;     // indices of the next tile
  template <typename BV, typename Sched>
  __device__ __forceinline__ void start(const BV& b, const Sched& sch) {
    nb = EdgeTileBounds{};
    nx = EdgeTileIdx{};
    if (sch.begin < sch.end) {
      EdgeTileBounds b0;
      b0.load(b, sch.begin);
      nx.load(b, b0);
    }
    if (sch.begin + sch.step < sch.end) nb.load(b, sch.begin + sch.step);
  }
  // After the current tile t has taken nx: issue the next tile's indices and
  // the bounds of the one after.
  template <typename BV, typename Sched>
  __device__ __forceinline__ void advance(const BV& b, const Sched& sch, int t) {
    if (t + sch.step < sch.end) nx.load(b, nb);
    if (t + 2 * sch.step < sch.end) nb.load(b, t + 2 * sch.step);
  }
};

// Segment starts of an edge tile, in LDS: seg[rl] is the first tile-local
// edge of receiver r0 + rl and seg[r1 - r0] = ne, so a receiver's edges are
// [seg[rl], seg[rl + 1]) (empty for a receiver without edges).  Derived from
// the receivers rs[0, ne) of the tile's edges (ascending, all in [r0, r1)),
// which must be visible in LDS, so the segment sums read no CSR row
// pointers from memory; each entry is written by exactly one thread (the
// edge at a receiver change, or the tile's last edge for the tail).
__device__ __forceinline__ void tile_segments(int* seg, const int* rs, int r0, int r1, int ne) {
  const int i = threadIdx.x;
  if (i < ne) {
    const int c = rs[i];
    for (int r = (i ? rs[i - 1] : r0 - 1) + 1; r <= c; ++r) seg[r - r0] = i;
  }
  if (i == (ne ? ne - 1 : 0))
    for (int r = (ne ? rs[ne - 1] : r0 - 1) + 1; r <= r1; ++r) seg[r - r0] = ne;
}

// Persistent-grid tile schedule.  The workgroups of the grid are dealt
// round-robin to the 8 XCDs (workgroup b runs on XCD b % 8); each XCD takes a
// contiguous eighth of the tiles so that neighbouring tiles, which share
// gathered node rows, meet in the same L2.  Tiles of an XCD are taken in
// order by its workgroups.  The mapping depends only on (n_tiles, grid), so
// the work of each workgroup -- and every partial sum -- is deterministic.
struct TileSched {
  int begin, end, step;
  __device__ TileSched(int n_tiles) {
    const int G = gridDim.x, b = blockIdx.x;
    const int x = b & 7, j = b >> 3;
    const int per_x = (G + 7 - x) >> 3;  // workgroups on XCD x
    const int t0 = (int)(((long long)n_tiles * x) >> 3);
    const int t1 = (int)(((long long)n_tiles * (x + 1)) >> 3);
    begin = t0 + j;
    end = t1;
    step = per_x;
  }
};

}  // namespace xmgn
