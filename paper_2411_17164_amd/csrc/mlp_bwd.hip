// Backward kernels: hand-written adjoints of the processor, encoders and
// decoder.  Every layer is recomputed from its checkpoint (h^l, e^l, m^l)
// inside the kernel (activation checkpointing), so only layer inputs are kept
// between forward and backward.
//
// Edge adjoint, for v = LN(u), u = W2 z + b2, z = act(a), a = W1 x + b1,
// x = [h_r ; h_s ; e]:
//   dv   = dm_r + de'_k                (v feeds m_r and the residual e')
//   du   = LN^T(dv),  dz = W2^T du,  da = dz * act'(a)
//   de_k = de'_k + (W1^T da)[2H:3H]     (plus dm_r when m sums e')
// The node-input parts of W1^T da are linear in da, so they are summed over
// edges first:  S_r = sum_{in(r)} da_k,  S_s = sum_{out(s)} da_k,
//   dh_r += W1_r^T S_r,  dh_s += W1_s^T S_s
// (the same value as summing W1^T da_k per edge, re-associated).  S_r is a
// tile-local segmented sum; S_s a sender-ordered (CSC) sum.  Weight
// gradients are row-sums of outer products and are formed by the wgrad
// kernel from the per-row factors written here; bias / LayerNorm gradients
// are per-workgroup column sums reduced in a fixed order.  No float atomics.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace xmgn {

template <typename T, int H, int NW = NWAVE>
struct BD {
  static constexpr int PAD = 16 / sizeof(T);
  static constexpr int LDH = H + PAD;
  static constexpr int LD2 = 2 * H + PAD;
  static constexpr int LD3 = 3 * H + PAD;
  static constexpr int LDF = H + 4;
  static constexpr int NB = H / (16 * NW);
  static constexpr int CPW = H / NW;
};

// Copy an FP32 [rows][H] block from global into an FP32 LDS tile (zero
// fill); NTHR threads, all loads issued before the stores.
template <int H, int LDF, int MT, typename SrcFn>
__device__ __forceinline__ void f32_rows_to_lds(float* dst, int rows, SrcFn src) {
  f32_tile<MT, H, NTHR>(
      rows, false, src, [](int, int) { return float4{0.f, 0.f, 0.f, 0.f}; },
      [&](int i, int q, const float4& v) { *(float4*)(dst + i * LDF + 4 * q) = v; });
}

template <int MB, int NB, int LDF>
__device__ __forceinline__ void acc_to_ldsf(const f32x4 (&x)[MB][NB], float* dst, int n0) {
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[acc_row(mb, r) * LDF + acc_col(n0, nb)] = x[mb][nb][r];
}

// LayerNorm adjoint in registers.  On entry xh = xhat, dv = upstream
// gradient (C layout); on exit dv holds du.  Accumulates dgamma, dbeta.
template <int MB, int NB, int MT, int H, int NW = NWAVE>
__device__ __forceinline__ void ln_backward(const f32x4 (&xh)[MB][NB], f32x4 (&dv)[MB][NB], const float (&inv)[MB][4],
                                            const float* gamma, int n0, float* red, double (&cg)[NB],
                                            double (&cbt)[NB]) {
  f32x4 gx[MB][NB];
  {
    f32x4 t[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) t[mb][nb][r] = dv[mb][nb][r] * xh[mb][nb][r];
    col_accumulate(t, cg);
  }
  col_accumulate(dv, cbt);
  // dv := g = dv * gamma ; gx = g * xhat
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const float gm = gamma[acc_col(n0, nb)];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        dv[mb][nb][r] *= gm;
        gx[mb][nb][r] = dv[mb][nb][r] * xh[mb][nb][r];
      }
    }
  float sg[MB][4], sgx[MB][4];
  row_sum2<MB, NB, MT, NW>(dv, gx, red, sg, sgx);
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        dv[mb][nb][r] = (dv[mb][nb][r] - sg[mb][r] * (1.f / H) - xh[mb][nb][r] * (sgx[mb][r] * (1.f / H))) * inv[mb][r];
}

// acc[nb][jb] += sum over the MT rows of a tile of
//   G[row][n0 + 16 nb + i] * B[row][16 jb + j],
// the rows n0 + 16 nb (this wave's columns of G) of a H x H weight gradient
// G^T B.  The A operand is the wave's own FP32 accumulator tile G, rounded
// to BF16: in the MFMA accumulator layout, lane group q holds rows
// 4q + r and 16 + 4q + r (r < 4) of each 32-row k chunk.  The order of k
// inside one MFMA is free, so B is read in that same row order from its
// row-major LDS tile (row stride LDB) with transposing reads.
template <int MB, int NB, int H, int LDB>
__device__ __forceinline__ void wave_wgrad(f32x4 (&acc)[NB][H / 16], const f32x4 (&g)[MB][NB], const bf16* B) {
  static_assert(MB % 2 == 0, "k chunks of 32 rows");
  const int lg = lane_id() >> 4;
#pragma unroll
  for (int c = 0; c < MB / 2; ++c) {
    bf16x8 a[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        a[nb][r] = (bf16)g[2 * c][nb][r];
        a[nb][4 + r] = (bf16)g[2 * c + 1][nb][r];
      }
#pragma unroll
    for (int jb = 0; jb < H / 16; ++jb) {
      const bf16x8 b = lds_bfrag_tr(B, LDB, 32 * c + 4 * lg, jb * 16, 16);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb][jb] = mma(a[nb], b, acc[nb][jb]);
    }
  }
}

template <int NB>
__device__ __forceinline__ void write_partial(float* p, int n0, const double (&v)[NB]) {
  if ((lane_id() >> 4) == 0)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) p[acc_col(n0, nb)] = (float)v[nb];
}

// ---------------------------------------------------------------------------
// Edge adjoint (with recompute).
// ---------------------------------------------------------------------------
// FW = 1 (BF16, H = 128): also accumulate dW2 = sum du z^T and the e-block
// of dW1 = sum da e^T per workgroup on MFMA -- du and da straight from the
// accumulators, z and e read transposed from their LDS tiles -- so that z
// and du never travel to HBM; partials go to o.wpart.  W2 and the e-block of
// W1 then live in LDS for the whole kernel and serve both their products and
// (read transposed) the adjoint products dz = du W2 and de = da W1e; the FP32
// staging tile takes the first 2H columns of the gathered tile's rows so that
// its e columns stay intact.  One workgroup per compute unit.
// FW = 2 (BF16, H = 128, z from the tape, 32-row tiles): dW2 only, W2 alone
// in LDS, the e-block of W1 read from L2 for de = da W1e, and the e-block of
// dW1 left to a separate product over da (which is written anyway) and the e
// tape.  Half the accumulator registers and under 80 KB of LDS: two
// workgroups per compute unit, so one's loads and barriers overlap the
// other's arithmetic.
template <typename T, int H, int MT, int FW, int NW>
struct EdgeBwdLds {
  using D = BD<T, H, NW>;
  static constexpr size_t XS = (size_t)MT * D::LD3 * sizeof(T);
  static constexpr size_t ZS = (size_t)MT * D::LDH * sizeof(T);
  static constexpr int LDW = H + 8;  // LDS-resident weights (BF16)
  static constexpr size_t WS = FW ? (size_t)H * LDW * 2 : 0;
  static constexpr int NWS = FW == 1 ? 2 : FW == 2 ? 1 : 0;  // LDS-resident weight matrices
  static constexpr int LDF = FW ? D::LD3 * (int)sizeof(T) / 4 : D::LDF;  // FP32 staging row stride
  // receivers, senders, segment starts (MT + 1, padded)
  static constexpr size_t bytes = XS + ZS + NWS * WS + 2 * NW * MT * 4 + (3 * MT + 4) * 4;
};

// ZT (BF16): z of every edge comes from the forward's tape (zt) instead of
// being recomputed -- no gather of h_r, h_s and no first product.  ReLU's
// derivative is [z > 0], exactly [a > 0]; SiLU's takes a from the tape of
// pre-activations (at, BF16).  Unfused (H = 256, 512), the dW2 product then
// reads z from the tape too.
template <typename T, int H, int MT, int ACT, int AGG, int FW, int NW, int ZT>
__global__ __launch_bounds__(64 * NW, waves_per_simd(EdgeBwdLds<T, H, MT, FW, NW>::bytes, NW)) void k_edge_bwd(
    BatchView b, MlpW w, const T* __restrict__ h, const T* __restrict__ e, const T* __restrict__ zt,
    const T* __restrict__ at, const float* __restrict__ de_in, const float* __restrict__ dm, EdgeBwdOut o,
    float eps) {
  using D = BD<T, H, NW>;
  using L = EdgeBwdLds<T, H, MT, FW, NW>;
  constexpr int MB = MT / 16, NB = D::NB;
  constexpr size_t XS = L::XS, ZS = L::ZS, WS = L::WS;
  constexpr int LDW = L::LDW, LDF = L::LDF;
  static_assert(!FW || (sizeof(T) == 2 && H == 128), "fused weight gradients: BF16, H = 128");
  static_assert(FW != 2 || ZT, "dW2-only fusion reads z from the tape");
  static_assert((size_t)MT * LDF * 4 <= XS, "FP32 tile must fit in the staging tile");
  static_assert(!FW || (size_t)H * 4 <= 2 * H * sizeof(T), "FP32 rows must leave the e columns intact");
  // z from the tape, fused weight gradients, ReLU: the FP32 tile's columns
  // are free from the start of a tile, so dv is loaded with z and e
  constexpr bool EARLY_DV = ZT && FW && ACT == 0;
  __shared__ __align__(16) unsigned char smem[L::bytes];
  T* xs = (T*)smem;
  float* ft = (float*)smem;
  T* zs = (T*)(smem + XS);
  bf16* W2s = (bf16*)(smem + XS + ZS);       // W2 [out][in]
  bf16* W1es = (bf16*)(smem + XS + ZS + WS);  // W1[:, 2H:3H] [out][in] (FW = 1)
  float* red = (float*)(smem + XS + ZS + L::NWS * WS);
  int* rs = (int*)(red + 2 * NW * MT);
  const T* W1 = (const T*)w.W1;
  const T* W2 = (const T*)w.W2;
  const T* W2T = (const T*)w.W2T;
  const T* W1Te = (const T*)w.W1T;
  const int n0 = wave_id() * D::CPW;
  const int li = lane_id() & 15, lg = lane_id() >> 4;
  double cb1[NB] = {}, cb2[NB] = {}, cg[NB] = {}, cbt[NB] = {};
  f32x4 accW2[NB][H / 16], accW1[NB][H / 16];
  if constexpr (FW) {
    zero_acc(accW2);
    if constexpr (FW == 1) zero_acc(accW1);
    // weights resident in LDS (visible after the first barrier of the tile loop)
    for (int c = threadIdx.x; c < H * (H / 8); c += 64 * NW) {
      const int r = c / (H / 8), q = c - r * (H / 8);
      *(uint4*)(W2s + r * LDW + 8 * q) = *(const uint4*)(W2 + (size_t)r * H + 8 * q);
      if constexpr (FW == 1)
        *(uint4*)(W1es + r * LDW + 8 * q) = *(const uint4*)(W1 + (size_t)r * 3 * H + 2 * H + 8 * q);
    }
  }

  TileSched sch(b.n_etiles);
  EdgeTileIdx nx{};  // a tile ahead; deeper prefetch costs this kernel registers it spills
  if (sch.begin < sch.end) nx.load(b, sch.begin);
  for (int t = sch.begin; t < sch.end; t += sch.step) {
    const EdgeTileIdx cur = nx;
    const int r0 = cur.r0, r1 = cur.r1, e0 = cur.e0, ne = cur.ne;
    int* ss = rs + MT;
    int* sg = rs + 2 * MT;
    if (threadIdx.x < MT) {
      rs[threadIdx.x] = cur.rv;
      ss[threadIdx.x] = cur.cv;
    }
    lds_sync();
    tile_segments(sg, rs, r0, r1, ne);  // read after the next barrier
    if constexpr (ZT) {
      // z rows into zs, (fused: for dW1's e-block) e rows into the e columns
      // of xs and (SiLU) a rows into its first H columns, one batch of loads
      constexpr int NPART = 1 + (FW == 1 ? 1 : 0) + (ACT != 0 ? 1 : 0);
      constexpr int E8 = 16 / sizeof(T), CPR = H / E8, TOT = NPART * MT * CPR, IT = TOT / (64 * NW);
      static_assert(TOT % (64 * NW) == 0, "whole steps of the workgroup");
      auto src = [&](int p) -> const T* { return p == 0 ? zt : (FW == 1 && p == 1) ? e : at; };
      auto dst = [&](int p, int i, int q) -> T* {
        return p == 0 ? zs + i * D::LDH + q * E8 : (FW == 1 && p == 1) ? xs + i * D::LD3 + 2 * H + q * E8
                                                                  : xs + i * D::LD3 + q * E8;
      };
      uint4 v[IT];
#pragma unroll
      for (int k = 0; k < IT; ++k) {
        const int c = (int)threadIdx.x + k * 64 * NW, p = c / (MT * CPR), rem = c - p * (MT * CPR);
        const int i = rem / CPR, q = rem - i * CPR;
        v[k] = uint4{0u, 0u, 0u, 0u};
        if (i < ne) v[k] = *(const uint4*)(src(p) + (size_t)(e0 + i) * H + q * E8);
      }
      if constexpr (EARLY_DV)  // dv = dm_r + de' in the same round trip, into the FP32 tile
        f32_tile<MT, H, 64 * NW>(
            ne, de_in != nullptr, [&](int i, int q) { return *(const float4*)(dm + (size_t)rs[i] * H + 4 * q); },
            [&](int i, int q) { return *(const float4*)(de_in + (size_t)(e0 + i) * H + 4 * q); },
            [&](int i, int q, const float4& w4) { *(float4*)(ft + i * LDF + 4 * q) = w4; });
#pragma unroll
      for (int k = 0; k < IT; ++k) {
        const int c = (int)threadIdx.x + k * 64 * NW, p = c / (MT * CPR), rem = c - p * (MT * CPR);
        const int i = rem / CPR, q = rem - i * CPR;
        *(uint4*)dst(p, i, q) = v[k];
      }
    } else {
      gather_tile<T, D::LD3, MT, 3, H, 64 * NW>(
          xs, ne,
          [&](int p, int i) { return p == 0 ? h + (size_t)rs[i] * H : p == 1 ? h + (size_t)ss[i] * H : e + (size_t)(e0 + i) * H; },
          [](int, int, int, const uint4&) {});
    }
    if (t + sch.step < sch.end) nx.load(b, t + sch.step);  // next tile's indices, in flight from here
    lds_sync();

    // recompute: a, z, u, xhat (ZT, ReLU: a holds z, whose sign is a's)
    f32x4 a[MB][NB];
    f32x4 x[MB][NB];
    zero_acc(a);
    if constexpr (ZT) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            a[mb][nb][r] = ACT == 0 ? to_f(zs[acc_row(mb, r) * D::LDH + acc_col(n0, nb)])
                                    : to_f(xs[acc_row(mb, r) * D::LD3 + acc_col(n0, nb)]);
    } else if constexpr (FW == 1) {
      wave_gemm<T, MB, NB, 2 * H, D::LD3>(a, xs, W1, 3 * H, n0);  // [h_r ; h_s] blocks from global
      wave_gemm_lds<MB, NB, H, D::LD3>(a, (const bf16*)xs + 2 * H, [&](int k, int nb) {
        return *(const bf16x8*)(W1es + (n0 + 16 * nb + li) * LDW + k + 8 * lg);
      });
    } else {
      wave_gemm<T, MB, NB, 3 * H, D::LD3>(a, xs, W1, 3 * H, n0);
    }
    if constexpr (!ZT) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const float bb = w.b1[acc_col(n0, nb)];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            a[mb][nb][r] += bb;
            x[mb][nb][r] = act_f<ACT>(a[mb][nb][r]);
          }
        }
      acc_to_lds<T, MB, NB, D::LDH>(x, zs, n0);
      lds_sync();
    }
    zero_acc(x);
    if constexpr (FW) {
      wave_gemm_lds<MB, NB, H, D::LDH>(x, (const bf16*)zs, [&](int k, int nb) {
        return *(const bf16x8*)(W2s + (n0 + 16 * nb + li) * LDW + k + 8 * lg);
      });
    } else {
      wave_gemm<T, MB, NB, H, D::LDH>(x, zs, W2, H, n0);
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float bb = w.b2[acc_col(n0, nb)];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[mb][nb][r] += bb;
      }
    float inv[MB][4];
    ln_normalize<MB, NB, MT, H, NW>(x, red, eps, inv);  // x = xhat

    // upstream gradient dv = dm_r + de'_k  (FP32 tile over the dead gather)
    if constexpr (!EARLY_DV)
      f32_tile<MT, H, 64 * NW>(
          ne, de_in != nullptr, [&](int i, int q) { return *(const float4*)(dm + (size_t)rs[i] * H + 4 * q); },
          [&](int i, int q) { return *(const float4*)(de_in + (size_t)(e0 + i) * H + 4 * q); },
          [&](int i, int q, const float4& v) { *(float4*)(ft + i * LDF + 4 * q) = v; });
    if constexpr (!FW && !ZT) lds_rows_to_global<T, D::LDH>(zs, ne, H, (T*)o.z + (size_t)e0 * H, H, [](int i) { return i; });
    lds_sync();
    f32x4 g[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) g[mb][nb][r] = ft[acc_row(mb, r) * LDF + acc_col(n0, nb)];
    ln_backward<MB, NB, MT, H, NW>(x, g, inv, w.gamma, n0, red, cg, cbt);  // g = du (barriers inside)
    col_accumulate(g, cb2);
    if constexpr (FW) {
      wave_wgrad<MB, NB, H, D::LDH>(accW2, g, (const bf16*)zs);  // dW2 += du^T z
      lds_sync();  // every wave is done reading z before du replaces it
    }
    acc_to_lds<T, MB, NB, D::LDH>(g, zs, n0);
    lds_sync();
    if constexpr (!FW) lds_rows_to_global<T, D::LDH>(zs, ne, H, (T*)o.du + (size_t)e0 * H, H, [](int i) { return i; });
    // dz = W2^T du ; da = dz * act'(a)
    zero_acc(x);
    if constexpr (FW) {
      wave_gemm_lds<MB, NB, H, D::LDH>(x, (const bf16*)zs, [&](int k, int nb) {
        return lds_bfrag_tr(W2s, LDW, k + 8 * lg, n0 + 16 * nb, 4);
      });
    } else {
      wave_gemm<T, MB, NB, H, D::LDH>(x, zs, W2T, H, n0);
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) x[mb][nb][r] *= act_d<ACT>(a[mb][nb][r]);
    col_accumulate(x, cb1);
    if constexpr (FW == 1) wave_wgrad<MB, NB, H, D::LD3>(accW1, x, (const bf16*)xs + 2 * H);  // dW1[:, 2H:3H] += da^T e
    lds_sync();
    acc_to_ldsf<MB, NB, LDF>(x, ft, n0);
    acc_to_lds<T, MB, NB, D::LDH>(x, zs, n0);
    lds_sync();
    // de' (+ dm_r) for de_out, in flight while S_r and the de product run
    constexpr int IT2 = MT * (H / 4) / (64 * NW);
    static_assert(MT * (H / 4) % (64 * NW) == 0, "whole steps of the workgroup");
    float4 dep[FW ? IT2 : 1];
    if constexpr (FW) {
#pragma unroll
      for (int k = 0; k < IT2; ++k) {
        const int c = (int)threadIdx.x + k * 64 * NW, i = c / (H / 4), q = c - i * (H / 4);
        float4 va = float4{0.f, 0.f, 0.f, 0.f}, vb = float4{0.f, 0.f, 0.f, 0.f};
        if (i < ne) {
          if (de_in) va = *(const float4*)(de_in + (size_t)(e0 + i) * H + 4 * q);
          if (AGG != 0) vb = *(const float4*)(dm + (size_t)rs[i] * H + 4 * q);
        }
        dep[k] = float4{va.x + vb.x, va.y + vb.y, va.z + vb.z, va.w + vb.w};
      }
    }
    // S_r: receiver-segment sums of da (FP32, ascending sender order)
    const int nr = r1 - r0;
    for (int task = threadIdx.x; task < nr * (H / 4); task += 64 * NW) {
      const int rl = task / (H / 4), q = task - rl * (H / 4);
      const int lo = sg[rl], hi = sg[rl + 1];
      float4 s = {0.f, 0.f, 0.f, 0.f};
      for (int i = lo; i < hi; ++i) {
        const float4 v = *(const float4*)(ft + i * LDF + 4 * q);
        s.x += v.x;
        s.y += v.y;
        s.z += v.z;
        s.w += v.w;
      }
      *(float4*)(o.S_r + (size_t)(r0 + rl) * H + 4 * q) = s;
    }
    lds_rows_to_global<T, D::LDH>(zs, ne, H, (T*)o.da + (size_t)e0 * H, H, [](int i) { return i; });
    // de = de' (+ dm_r) + (W1^T da)[2H:3H]
    zero_acc(g);
    if constexpr (FW == 1) {
      wave_gemm_lds<MB, NB, H, D::LDH>(g, (const bf16*)zs, [&](int k, int nb) {
        return lds_bfrag_tr(W1es, LDW, k + 8 * lg, n0 + 16 * nb, 4);
      });
    } else {
      wave_gemm<T, MB, NB, H, D::LDH>(g, zs, W1Te, H, n0);
    }
    lds_sync();
    acc_to_ldsf<MB, NB, LDF>(g, ft, n0);
    lds_sync();
    if constexpr (FW) {
#pragma unroll
      for (int k = 0; k < IT2; ++k) {
        const int c = (int)threadIdx.x + k * 64 * NW, i = c / (H / 4), q = c - i * (H / 4);
        if (i < ne) {
          const float4 d = *(const float4*)(ft + i * LDF + 4 * q), v = dep[k];
          *(float4*)(o.de_out + (size_t)(e0 + i) * H + 4 * q) = float4{d.x + v.x, d.y + v.y, d.z + v.z, d.w + v.w};
        }
      }
    } else {
      f32_tile<MT, H, 64 * NW>(
          ne, AGG != 0, [&](int i, int q) { return de_in ? *(const float4*)(de_in + (size_t)(e0 + i) * H + 4 * q) : float4{0.f, 0.f, 0.f, 0.f}; },
          [&](int i, int q) { return *(const float4*)(dm + (size_t)rs[i] * H + 4 * q); },
          [&](int i, int q, const float4& v) {
            if (i < ne) {
              const float4 d = *(const float4*)(ft + i * LDF + 4 * q);
              *(float4*)(o.de_out + (size_t)(e0 + i) * H + 4 * q) = float4{d.x + v.x, d.y + v.y, d.z + v.z, d.w + v.w};
            }
          });
    }
    lds_sync();
  }
  float* p = o.partial + (size_t)blockIdx.x * 4 * H;
  write_partial<NB>(p, n0, cb1);
  write_partial<NB>(p + H, n0, cb2);
  write_partial<NB>(p + 2 * H, n0, cg);
  write_partial<NB>(p + 3 * H, n0, cbt);
  if constexpr (FW) {
    float* q2 = o.wpart + (size_t)blockIdx.x * 2 * H * H;
    float* q1 = q2 + H * H;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int jb = 0; jb < H / 16; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = n0 + nb * 16 + lg * 4 + r, n = jb * 16 + li;
          q2[m * H + n] = accW2[nb][jb][r];
          if constexpr (FW == 1) q1[m * H + n] = accW1[nb][jb][r];
        }
  }
}

// ---------------------------------------------------------------------------
// Node adjoint (with recompute).  dh_mid = dh' + (W1^T da)[0:H], dm = (W1^T da)[H:2H].
// FM (BF16, H = 128, 32-row tiles): W2 lives in LDS for the whole kernel
// and serves both its product and, read transposed, dz = du W2; dW2 is
// accumulated per workgroup on MFMA (du from the accumulators, z read
// transposed from its tile; partials to o.wpart [grid][H][H]), so z and du
// are not written.  78 KB of LDS: two workgroups per CU.  W1 and W1^T come
// from L2, and da is written for the two dW1 blocks, which are separate
// products over da, h and m.  (Keeping W1 in LDS too and fusing both dW1
// blocks takes 146 KB, one workgroup per CU, and measured slower.)
// ---------------------------------------------------------------------------
bool node_bwd_fuses_wgrad(const Shape& s) { return s.prec == 1 && s.H == 128 && s.mt_node == 32; }

template <typename T, int H, int MT, int ACT>
__global__ __launch_bounds__(NTHR, (MT == 32 && H == 128 ? 2 : 1)) void k_node_bwd(
    int n, MlpW w, const T* __restrict__ h, const float* __restrict__ m, const float* __restrict__ dh_in,
    NodeBwdOut o, float eps) {
  using D = BD<T, H>;
  constexpr bool FM = sizeof(T) == 2 && H == 128 && MT == 32;
  constexpr int MB = MT / 16, NB = D::NB;
  constexpr int LDW2 = H + 8;
  constexpr size_t XS = (size_t)MT * D::LD2 * sizeof(T);
  constexpr size_t ZS = (size_t)MT * D::LDH * sizeof(T);
  constexpr size_t W2S = FM ? (size_t)H * LDW2 * 2 : 0;
  static_assert((size_t)MT * D::LDF * 4 <= XS, "FP32 tile must fit in the staging tile");
  static_assert(!FM || MB % 2 == 0, "fused weight gradients: k chunks of 32 rows");
  __shared__ __align__(16) unsigned char smem[XS + ZS + 2 * NWAVE * MT * 4 + W2S];
  T* xs = (T*)smem;
  T* zs = (T*)(smem + XS);
  float* red = (float*)(smem + XS + ZS);
  bf16* W2s = (bf16*)(red + 2 * NWAVE * MT);  // FM: W2 [out][in]
  float* ft = (float*)smem;                   // aliases [h ; m] once the first product is done
  const T* W1 = (const T*)w.W1;
  const T* W2 = (const T*)w.W2;
  const T* W2T = (const T*)w.W2T;
  const T* W1T = (const T*)w.W1T;
  const int n0 = wave_id() * D::CPW;
  const int li = lane_id() & 15, lg = lane_id() >> 4;
  double cb1[NB] = {}, cb2[NB] = {}, cg[NB] = {}, cbt[NB] = {};
  f32x4 accW2[NB][H / 16];
  if constexpr (FM) {
    zero_acc(accW2);
    for (int c = threadIdx.x; c < H * (H / 8); c += NTHR) {
      const int r = c / (H / 8), q = c - r * (H / 8);
      *(uint4*)(W2s + r * LDW2 + 8 * q) = *(const uint4*)(W2 + (size_t)r * H + 8 * q);
    }
  }
  const int n_tiles = (n + MT - 1) / MT;
  // fused form, ReLU: the next tile's h and m rows travel in registers while
  // this tile computes, and this tile's dh_in rows are issued at its start,
  // so no HBM round trip waits on a tile's critical path (SiLU and the
  // unfused forms have no registers to spare: they would spill)
  constexpr bool PF = FM && ACT == 0;
  constexpr int CPF = H / 4, IF = PF ? MT * CPF / NTHR : 1;
  NodeRowsPre<T, H, MT, D::LD2> pre;  // (unused by the unfused forms)
  float4 pd[IF];

  TileSched sch(n_tiles);
  if constexpr (PF)
    if (sch.begin < sch.end) pre.load(h, m, sch.begin * MT, min(MT, n - sch.begin * MT));
  for (int t = sch.begin; t < sch.end; t += sch.step) {
    const int row0 = t * MT, nr = min(MT, n - row0);
    if constexpr (PF) {
#pragma unroll
      for (int k = 0; k < IF; ++k) {
        const int c = (int)threadIdx.x + k * NTHR, i = c / CPF, q = c - i * CPF;
        pd[k] = float4{0.f, 0.f, 0.f, 0.f};
        if (i < nr) pd[k] = *(const float4*)(dh_in + (size_t)(row0 + i) * H + 4 * q);
      }
      pre.store(xs);
      if (t + sch.step < sch.end) pre.load(h, m, (t + sch.step) * MT, min(MT, n - (t + sch.step) * MT));
    } else {
      global_rows_to_lds<T, D::LD2, MT, H>(xs, nr, 0, [&](int i) { return h + (size_t)(row0 + i) * H; });
      global_f32_rows_to_lds<T, D::LD2, MT, H>(xs, nr, H, [&](int i) { return m + (size_t)(row0 + i) * H; });
    }
    lds_sync();
    f32x4 a[MB][NB], x[MB][NB];
    zero_acc(a);
    wave_gemm<T, MB, NB, 2 * H, D::LD2>(a, xs, W1, 2 * H, n0);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float bb = w.b1[acc_col(n0, nb)];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          a[mb][nb][r] += bb;
          x[mb][nb][r] = act_f<ACT>(a[mb][nb][r]);
        }
      }
    acc_to_lds<T, MB, NB, D::LDH>(x, zs, n0);
    lds_sync();
    zero_acc(x);
    if constexpr (FM) {
      wave_gemm_lds<MB, NB, H, D::LDH>(x, (const bf16*)zs, [&](int k, int nb) {
        return *(const bf16x8*)(W2s + (n0 + 16 * nb + li) * LDW2 + k + 8 * lg);
      });
    } else {
      wave_gemm<T, MB, NB, H, D::LDH>(x, zs, W2, H, n0);
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float bb = w.b2[acc_col(n0, nb)];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[mb][nb][r] += bb;
      }
    float inv[MB][4];
    ln_normalize<MB, NB, MT, H>(x, red, eps, inv);
    if constexpr (PF) {
#pragma unroll
      for (int k = 0; k < IF; ++k) {
        const int c = (int)threadIdx.x + k * NTHR, i = c / CPF, q = c - i * CPF;
        *(float4*)(ft + i * D::LDF + 4 * q) = pd[k];
      }
    } else {
      f32_rows_to_lds<H, D::LDF, MT>(ft, nr, [&](int i, int q) { return *(const float4*)(dh_in + (size_t)(row0 + i) * H + 4 * q); });
    }
    if constexpr (!FM) lds_rows_to_global<T, D::LDH>(zs, nr, H, (T*)o.z + (size_t)row0 * H, H, [](int i) { return i; });
    lds_sync();
    f32x4 g[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) g[mb][nb][r] = ft[acc_row(mb, r) * D::LDF + acc_col(n0, nb)];
    ln_backward<MB, NB, MT, H>(x, g, inv, w.gamma, n0, red, cg, cbt);
    col_accumulate(g, cb2);
    if constexpr (FM) {
      wave_wgrad<MB, NB, H, D::LDH>(accW2, g, (const bf16*)zs);  // dW2 += du^T z
      lds_sync();  // every wave is done reading z before du replaces it
    }
    acc_to_lds<T, MB, NB, D::LDH>(g, zs, n0);
    lds_sync();
    zero_acc(x);
    if constexpr (FM) {
      wave_gemm_lds<MB, NB, H, D::LDH>(x, (const bf16*)zs, [&](int k, int nb) {
        return lds_bfrag_tr(W2s, LDW2, k + 8 * lg, n0 + 16 * nb, 4);
      });
    } else {
      lds_rows_to_global<T, D::LDH>(zs, nr, H, (T*)o.du + (size_t)row0 * H, H, [](int i) { return i; });
      wave_gemm<T, MB, NB, H, D::LDH>(x, zs, W2T, H, n0);
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) x[mb][nb][r] *= act_d<ACT>(a[mb][nb][r]);
    col_accumulate(x, cb1);
    lds_sync();
    acc_to_lds<T, MB, NB, D::LDH>(x, zs, n0);
    lds_sync();
    // da for the dW1 products
    lds_rows_to_global<T, D::LDH>(zs, nr, H, (T*)o.da + (size_t)row0 * H, H, [](int i) { return i; });
    zero_acc(g);
    zero_acc(x);
    wave_gemm<T, MB, NB, H, D::LDH>(g, zs, W1T, H, n0);                  // -> dh part
    wave_gemm<T, MB, NB, H, D::LDH>(x, zs, W1T + (size_t)H * H, H, n0);  // -> dm
    acc_to_ldsf<MB, NB, D::LDF>(g, ft, n0);
    lds_sync();
    f32_tile<MT, H, NTHR>(
        nr, false, [&](int i, int q) { return *(const float4*)(dh_in + (size_t)(row0 + i) * H + 4 * q); },
        [](int, int) { return float4{0.f, 0.f, 0.f, 0.f}; },
        [&](int i, int q, const float4& d) {
          if (i < nr) {
            const float4 v = *(const float4*)(ft + i * D::LDF + 4 * q);
            *(float4*)(o.dh_mid + (size_t)(row0 + i) * H + 4 * q) = float4{v.x + d.x, v.y + d.y, v.z + d.z, v.w + d.w};
          }
        });
    lds_sync();
    acc_to_ldsf<MB, NB, D::LDF>(x, ft, n0);
    lds_sync();
    for (int c = threadIdx.x; c < nr * (H / 4); c += NTHR) {
      const int i = c / (H / 4), q = c - i * (H / 4);
      *(float4*)(o.dm + (size_t)(row0 + i) * H + 4 * q) = *(const float4*)(ft + i * D::LDF + 4 * q);
    }
    lds_sync();
  }
  float* p = o.partial + (size_t)blockIdx.x * 4 * H;
  write_partial<NB>(p, n0, cb1);
  write_partial<NB>(p + H, n0, cb2);
  write_partial<NB>(p + 2 * H, n0, cg);
  write_partial<NB>(p + 3 * H, n0, cbt);
  if constexpr (FM) {
    float* q2 = o.wpart + (size_t)blockIdx.x * H * H;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int jb = 0; jb < H / 16; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) q2[(n0 + nb * 16 + lg * 4 + r) * H + jb * 16 + li] = accW2[nb][jb][r];
  }
}

// dh_out = dh_mid + [S_r | S_s] B_rs^T, B_rs = [W1_r^T | W1_s^T] ([H][2H]).
template <typename T, int H, int MT>
__global__ __launch_bounds__(NTHR, H == 128 ? 2 : 1) void k_node_dh(int n, const T* __restrict__ Brs, const float* __restrict__ dh_mid,
                                                  const float* __restrict__ S_r, const float* __restrict__ S_s,
                                                  float* __restrict__ dh_out) {
  using D = BD<T, H>;
  constexpr int MB = MT / 16, NB = D::NB;
  constexpr size_t XS = (size_t)MT * D::LD2 * sizeof(T);
  __shared__ __align__(16) unsigned char smem[XS + (size_t)MT * D::LDF * 4];
  T* xs = (T*)smem;
  float* ft = (float*)(smem + XS);
  const int n0 = wave_id() * D::CPW;
  const int n_tiles = (n + MT - 1) / MT;
  TileSched sch(n_tiles);
  for (int t = sch.begin; t < sch.end; t += sch.step) {
    const int row0 = t * MT, nr = min(MT, n - row0);
    global_f32_rows_to_lds<T, D::LD2, MT, H>(xs, nr, 0, [&](int i) { return S_r + (size_t)(row0 + i) * H; });
    global_f32_rows_to_lds<T, D::LD2, MT, H>(xs, nr, H, [&](int i) { return S_s + (size_t)(row0 + i) * H; });
    lds_sync();
    f32x4 acc[MB][NB];
    zero_acc(acc);
    wave_gemm<T, MB, NB, 2 * H, D::LD2>(acc, xs, Brs, 2 * H, n0);
    acc_to_ldsf<MB, NB, D::LDF>(acc, ft, n0);
    lds_sync();
    f32_tile<MT, H, NTHR>(
        nr, false, [&](int i, int q) { return *(const float4*)(dh_mid + (size_t)(row0 + i) * H + 4 * q); },
        [](int, int) { return float4{0.f, 0.f, 0.f, 0.f}; },
        [&](int i, int q, const float4& d) {
          if (i < nr) {
            const float4 v = *(const float4*)(ft + i * D::LDF + 4 * q);
            *(float4*)(dh_out + (size_t)(row0 + i) * H + 4 * q) = float4{v.x + d.x, v.y + d.y, v.z + d.z, v.w + d.w};
          }
        });
    lds_sync();
  }
}

// S_s[s] = sum over the out-edges of s (CSC order: ascending receiver) of da.
// A sender's row is covered by LPR lanes holding 16 bytes each; a wave takes
// 64 / LPR senders at once, and the edge loop is unrolled so several row
// loads are in flight.  Every lane adds its columns in CSC order.
template <typename T, int H>
__global__ __launch_bounds__(NTHR) void k_sender_sum(int n, const int* __restrict__ csc_ptr, const int* __restrict__ csc_edge,
                                                     const T* __restrict__ da, float* __restrict__ S_s) {
  constexpr int E = 16 / sizeof(T);   // elements per lane
  constexpr int LPR = H / E;          // lanes per row
  constexpr int SPW = 64 / LPR;       // senders per wave
  static_assert(LPR <= 64 && 64 % LPR == 0, "row must map onto a wave");
  const int l = lane_id();
  const int sub = l / LPR, q = l - sub * LPR;
  const int nw = gridDim.x * NWAVE;
  for (int s0 = (blockIdx.x * NWAVE + wave_id()) * SPW; s0 < n; s0 += nw * SPW) {
    const int s = s0 + sub;
    float acc[E];
#pragma unroll
    for (int c = 0; c < E; ++c) acc[c] = 0.f;
    if (s < n) {
      const int lo = csc_ptr[s], hi = csc_ptr[s + 1];
#pragma unroll 4
      for (int j = lo; j < hi; ++j) {
        const uint4 v = *(const uint4*)(da + (size_t)csc_edge[j] * H + q * E);
        const T* pv = (const T*)&v;
#pragma unroll
        for (int c = 0; c < E; ++c) acc[c] += to_f(pv[c]);
      }
      float* dst = S_s + (size_t)s * H + q * E;
#pragma unroll
      for (int c = 0; c < E; c += 4) *(float4*)(dst + c) = make_float4(acc[c], acc[c + 1], acc[c + 2], acc[c + 3]);
    }
  }
}

// ---------------------------------------------------------------------------
// Decoder adjoint on inner rows: dy -> dz2 = W3^T dy, da2, dz1 = W2^T da2,
// da1, dh = W1^T da1.  Writes the factors of the weight gradients.
// ---------------------------------------------------------------------------
template <typename T, int H, int MT, int ACT>
__global__ __launch_bounds__(NTHR, H == 128 ? 2 : 1) void k_dec_bwd(BatchView b, MlpW w, const T* __restrict__ h,
                                                  const float* __restrict__ d_out, int out_dim, DecBwdOut o) {
  using D = BD<T, H>;
  constexpr int MB = MT / 16, NB = D::NB;
  constexpr size_t ZS = (size_t)MT * D::LDH * sizeof(T);
  constexpr size_t FS = (size_t)MT * D::LDF * 4;
  __shared__ __align__(16) unsigned char smem[3 * ZS + FS + MT * 16 * 4];
  T* xs = (T*)smem;
  T* zs = (T*)(smem + ZS);
  T* z2s = (T*)(smem + 2 * ZS);
  float* ft = (float*)(smem + 3 * ZS);
  float* dys = (float*)(smem + 3 * ZS + FS);
  const T* W1 = (const T*)w.W1;
  const T* W2 = (const T*)w.W2;
  const T* W1T = (const T*)w.W1T;
  const T* W2T = (const T*)w.W2T;
  const float* W3 = w.W1f;
  const int n0 = wave_id() * D::CPW;
  double cb1[NB] = {}, cb2[NB] = {};
  double cb3 = 0.0;
  const int n_tiles = (b.n_inner + MT - 1) / MT;

  TileSched sch(n_tiles);
  for (int t = sch.begin; t < sch.end; t += sch.step) {
    const int row0 = t * MT, nr = min(MT, b.n_inner - row0);
    global_rows_to_lds<T, D::LDH, MT, H>(xs, nr, 0, [&](int i) { return h + (size_t)b.inner[row0 + i] * H; });
    for (int c = threadIdx.x; c < MT * 16; c += NTHR) {
      const int i = c >> 4, oo = c & 15;
      dys[c] = (i < nr && oo < out_dim) ? d_out[(size_t)b.gid[b.inner[row0 + i]] * out_dim + oo] : 0.f;
    }
    lds_sync();
    if ((int)threadIdx.x < out_dim)
      for (int i = 0; i < nr; ++i) cb3 += dys[i * 16 + threadIdx.x];
    f32x4 a1[MB][NB], a2[MB][NB], x[MB][NB];
    zero_acc(a1);
    wave_gemm<T, MB, NB, H, D::LDH>(a1, xs, W1, H, n0);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float bb = w.b1[acc_col(n0, nb)];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          a1[mb][nb][r] += bb;
          x[mb][nb][r] = act_f<ACT>(a1[mb][nb][r]);
        }
      }
    acc_to_lds<T, MB, NB, D::LDH>(x, zs, n0);
    lds_sync();
    zero_acc(a2);
    wave_gemm<T, MB, NB, H, D::LDH>(a2, zs, W2, H, n0);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int c = acc_col(n0, nb);
        const float bb = w.b2[c];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          a2[mb][nb][r] += bb;
          x[mb][nb][r] = act_f<ACT>(a2[mb][nb][r]);
          const float* dy = dys + acc_row(mb, r) * 16;
          float dz = 0.f;
          for (int oo = 0; oo < out_dim; ++oo) dz += dy[oo] * W3[oo * H + c];
          a2[mb][nb][r] = dz * act_d<ACT>(a2[mb][nb][r]);  // a2 := da2
        }
      }
    col_accumulate(a2, cb2);
    acc_to_lds<T, MB, NB, D::LDH>(x, z2s, n0);
    lds_sync();
    lds_rows_to_global<T, D::LDH>(z2s, nr, H, (T*)o.z2 + (size_t)row0 * H, H, [](int i) { return i; });
    lds_rows_to_global<T, D::LDH>(zs, nr, H, (T*)o.z1 + (size_t)row0 * H, H, [](int i) { return i; });
    for (int c = threadIdx.x; c < nr * 16; c += NTHR) o.dy[(size_t)row0 * 16 + c] = dys[c];
    lds_sync();
    acc_to_lds<T, MB, NB, D::LDH>(a2, z2s, n0);
    lds_sync();
    lds_rows_to_global<T, D::LDH>(z2s, nr, H, (T*)o.da2 + (size_t)row0 * H, H, [](int i) { return i; });
    zero_acc(x);
    wave_gemm<T, MB, NB, H, D::LDH>(x, z2s, W2T, H, n0);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) x[mb][nb][r] *= act_d<ACT>(a1[mb][nb][r]);
    col_accumulate(x, cb1);
    lds_sync();
    acc_to_lds<T, MB, NB, D::LDH>(x, z2s, n0);
    lds_sync();
    lds_rows_to_global<T, D::LDH>(z2s, nr, H, (T*)o.da1 + (size_t)row0 * H, H, [](int i) { return i; });
    zero_acc(x);
    wave_gemm<T, MB, NB, H, D::LDH>(x, z2s, W1T, H, n0);
    acc_to_ldsf<MB, NB, D::LDF>(x, ft, n0);
    lds_sync();
    for (int c = threadIdx.x; c < nr * (H / 4); c += NTHR) {
      const int i = c / (H / 4), q = c - i * (H / 4);
      *(float4*)(o.dh + (size_t)b.inner[row0 + i] * H + 4 * q) = *(const float4*)(ft + i * D::LDF + 4 * q);
    }
    lds_sync();
  }
  float* p = o.partial + (size_t)blockIdx.x * (2 * H + 16);
  write_partial<NB>(p, n0, cb1);
  write_partial<NB>(p + H, n0, cb2);
  if (threadIdx.x < 16) p[2 * H + threadIdx.x] = (int)threadIdx.x < out_dim ? (float)cb3 : 0.f;
}

// ---------------------------------------------------------------------------
// Encoder adjoint: y = LN(W3 act(W2 act(W1 x + b1) + b2) + b3).  dW1
// (H x in) is accumulated per workgroup since in <= 8.  dW3 and dW2 are
// either accumulated per workgroup on MFMA as well (FE: BF16, H = 128 --
// du3 and da2 straight from the accumulators, z2 and z1 read transposed from
// their LDS tiles, W2 and W3 resident in LDS and read transposed for the
// adjoint products; partials go to o.wpart), or du3, z2, da2, z1 are
// written out for separate weight-gradient products.
// ---------------------------------------------------------------------------
bool enc_bwd_fuses_wgrad(const Shape& s) { return s.prec == 1 && s.H == 128; }

// KIN as for k_enc_fwd; with 32 input slots the input layer's dW1 is left to
// a separate product over o.da1 (its FP32 adjoint, written here).
template <typename T, int H, int MT, int ACT, int KIND, int KIN>
__global__ __launch_bounds__(NTHR) void k_enc_bwd(int rows, BatchView b, MlpW w, const float* __restrict__ src, int in_dim,
                                                  const float* __restrict__ dout, EncBwdOut o, float eps) {
  using D = BD<T, H>;
  constexpr bool FE = sizeof(T) == 2 && H == 128;
  constexpr int MB = MT / 16, NB = D::NB;
  constexpr int LDW = H + 8;
  constexpr size_t ZS = (size_t)MT * D::LDH * sizeof(T);
  constexpr size_t FS = (size_t)MT * D::LDF * 4;
  constexpr size_t WS = FE ? (size_t)H * LDW * 2 : 0;
  static_assert(!FE || (MB % 2 == 0 && ZS <= FS), "fused weight gradients: k chunks of 32 rows, du3 over the FP32 tile");
  __shared__ __align__(16) unsigned char smem[2 * ZS + FS + MT * KIN * 4 + 2 * NWAVE * MT * 4 + 2 * WS];
  T* zs = (T*)smem;
  T* z2s = (T*)(smem + ZS);
  float* ft = (float*)(smem + 2 * ZS);
  T* du3s = (T*)ft;  // FE: du3 once the FP32 tile is dead
  float* xin = (float*)(smem + 2 * ZS + FS);
  float* red = xin + MT * KIN;  // [2][NWAVE][MT]
  bf16* W2s = (bf16*)(red + 2 * NWAVE * MT);  // FE: W2 [out][in]
  bf16* W3s = W2s + (FE ? H * LDW : 0);       // FE: W3 [out][in]
  const T* W2 = (const T*)w.W2;
  const T* W3 = (const T*)w.W3;
  const T* W2T = (const T*)w.W2T;
  const T* W3T = (const T*)w.W3T;
  const int n0 = wave_id() * D::CPW;
  const int li = lane_id() & 15, lg = lane_id() >> 4;
  double cb1[NB] = {}, cb2[NB] = {}, cb3[NB] = {}, cg[NB] = {}, cbt[NB] = {};
  double cw1[NB][KIN == 8 ? 8 : 1] = {};
  f32x4 accW2[NB][H / 16], accW3[NB][H / 16];
  if constexpr (FE) {
    zero_acc(accW2);
    zero_acc(accW3);
    for (int c = threadIdx.x; c < H * (H / 8); c += NTHR) {
      const int r = c / (H / 8), q = c - r * (H / 8);
      *(uint4*)(W2s + r * LDW + 8 * q) = *(const uint4*)(W2 + (size_t)r * H + 8 * q);
      *(uint4*)(W3s + r * LDW + 8 * q) = *(const uint4*)(W3 + (size_t)r * H + 8 * q);
    }
  }
  const int n_tiles = (rows + MT - 1) / MT;

  TileSched sch(n_tiles);
  for (int t = sch.begin; t < sch.end; t += sch.step) {
    const int row0 = t * MT, nr = min(MT, rows - row0);
    if constexpr (KIN == 8) {
      if (threadIdx.x < MT) {
        const int i = threadIdx.x;
        float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (i < nr) {
          if constexpr (KIND == 0) {
            const float* p = src + (size_t)b.gid[row0 + i] * in_dim;
            for (int k = 0; k < in_dim; ++k) v[k] = p[k];
          } else {
            const float4 f = ((const float4*)src)[row0 + i];  // edge features (k_edge_feat)
            v[0] = f.x;
            v[1] = f.y;
            v[2] = f.z;
            v[3] = f.w;
          }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) xin[i * 8 + k] = v[k];
      }
    } else {
      for (int task = threadIdx.x; task < MT * KIN; task += NTHR) {
        const int i = task / KIN, k = task - i * KIN;
        xin[task] = (i < nr && k < in_dim) ? src[(size_t)b.gid[row0 + i] * in_dim + k] : 0.f;
      }
    }
    lds_sync();
    f32x4 a1[MB][NB], a2[MB][NB], x[MB][NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int c = acc_col(n0, nb);
      const float bb = w.b1[c];
      if constexpr (KIN == 8) {
        float wr[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) wr[k] = k < in_dim ? w.W1f[c * in_dim + k] : 0.f;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float* xi = xin + acc_row(mb, r) * 8;
            float s = bb;
#pragma unroll
            for (int k = 0; k < 8; ++k) s += wr[k] * xi[k];
            a1[mb][nb][r] = s;
          }
      } else {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int r = 0; r < 4; ++r) a1[mb][nb][r] = bb;
        for (int k = 0; k < in_dim; ++k) {
          const float wk = w.W1f[c * in_dim + k];
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int r = 0; r < 4; ++r) a1[mb][nb][r] += wk * xin[acc_row(mb, r) * KIN + k];
        }
      }
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int r = 0; r < 4; ++r) x[mb][nb][r] = act_f<ACT>(a1[mb][nb][r]);
    }
    acc_to_lds<T, MB, NB, D::LDH>(x, zs, n0);
    lds_sync();
    zero_acc(a2);
    if constexpr (FE) {
      wave_gemm_lds<MB, NB, H, D::LDH>(a2, (const bf16*)zs, [&](int k, int nb) {
        return *(const bf16x8*)(W2s + (n0 + 16 * nb + li) * LDW + k + 8 * lg);
      });
    } else {
      wave_gemm<T, MB, NB, H, D::LDH>(a2, zs, W2, H, n0);
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float bb = w.b2[acc_col(n0, nb)];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          a2[mb][nb][r] += bb;
          x[mb][nb][r] = act_f<ACT>(a2[mb][nb][r]);
        }
      }
    acc_to_lds<T, MB, NB, D::LDH>(x, z2s, n0);
    lds_sync();
    zero_acc(x);
    if constexpr (FE) {
      wave_gemm_lds<MB, NB, H, D::LDH>(x, (const bf16*)z2s, [&](int k, int nb) {
        return *(const bf16x8*)(W3s + (n0 + 16 * nb + li) * LDW + k + 8 * lg);
      });
    } else {
      wave_gemm<T, MB, NB, H, D::LDH>(x, z2s, W3, H, n0);
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float bb = w.b3[acc_col(n0, nb)];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[mb][nb][r] += bb;
      }
    float inv[MB][4];
    ln_normalize<MB, NB, MT, H>(x, red, eps, inv);
    f32_rows_to_lds<H, D::LDF, MT>(ft, nr, [&](int i, int q) { return *(const float4*)(dout + (size_t)(row0 + i) * H + 4 * q); });
    if constexpr (!FE) {
      lds_rows_to_global<T, D::LDH>(zs, nr, H, (T*)o.z1 + (size_t)row0 * H, H, [](int i) { return i; });
      lds_rows_to_global<T, D::LDH>(z2s, nr, H, (T*)o.z2 + (size_t)row0 * H, H, [](int i) { return i; });
    }
    lds_sync();
    f32x4 g[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) g[mb][nb][r] = ft[acc_row(mb, r) * D::LDF + acc_col(n0, nb)];
    ln_backward<MB, NB, MT, H>(x, g, inv, w.gamma, n0, red, cg, cbt);  // barriers inside: ft is dead after
    col_accumulate(g, cb3);
    zero_acc(x);
    if constexpr (FE) {
      wave_wgrad<MB, NB, H, D::LDH>(accW3, g, (const bf16*)z2s);  // dW3 += du3^T z2
      acc_to_lds<T, MB, NB, D::LDH>(g, du3s, n0);
      lds_sync();
      wave_gemm_lds<MB, NB, H, D::LDH>(x, (const bf16*)du3s, [&](int k, int nb) {
        return lds_bfrag_tr(W3s, LDW, k + 8 * lg, n0 + 16 * nb, 4);
      });
    } else {
      acc_to_lds<T, MB, NB, D::LDH>(g, zs, n0);
      lds_sync();
      lds_rows_to_global<T, D::LDH>(zs, nr, H, (T*)o.du3 + (size_t)row0 * H, H, [](int i) { return i; });
      wave_gemm<T, MB, NB, H, D::LDH>(x, zs, W3T, H, n0);
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) x[mb][nb][r] *= act_d<ACT>(a2[mb][nb][r]);
    col_accumulate(x, cb2);
    if constexpr (FE) wave_wgrad<MB, NB, H, D::LDH>(accW2, x, (const bf16*)zs);  // dW2 += da2^T z1
    lds_sync();
    acc_to_lds<T, MB, NB, D::LDH>(x, z2s, n0);
    lds_sync();
    zero_acc(x);
    if constexpr (FE) {
      wave_gemm_lds<MB, NB, H, D::LDH>(x, (const bf16*)z2s, [&](int k, int nb) {
        return lds_bfrag_tr(W2s, LDW, k + 8 * lg, n0 + 16 * nb, 4);
      });
    } else {
      lds_rows_to_global<T, D::LDH>(z2s, nr, H, (T*)o.da2 + (size_t)row0 * H, H, [](int i) { return i; });
      wave_gemm<T, MB, NB, H, D::LDH>(x, z2s, W2T, H, n0);
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) x[mb][nb][r] *= act_d<ACT>(a1[mb][nb][r]);
    col_accumulate(x, cb1);
    if constexpr (KIN == 8) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          float s = 0.f;
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int r = 0; r < 4; ++r) s += x[mb][nb][r] * xin[acc_row(mb, r) * 8 + k];
          cw1[nb][k] += (double)sum_groups(s);
        }
    } else {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = acc_row(mb, r);
            if (row < nr) o.da1[(size_t)(row0 + row) * H + acc_col(n0, nb)] = x[mb][nb][r];
          }
    }
    lds_sync();
  }
  float* p = o.partial + (size_t)blockIdx.x * 13 * H;
  write_partial<NB>(p, n0, cb1);
  write_partial<NB>(p + H, n0, cb2);
  write_partial<NB>(p + 2 * H, n0, cb3);
  write_partial<NB>(p + 3 * H, n0, cg);
  write_partial<NB>(p + 4 * H, n0, cbt);
  if constexpr (KIN == 8)
    if ((lane_id() >> 4) == 0)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int k = 0; k < 8; ++k) p[5 * H + acc_col(n0, nb) * 8 + k] = (float)cw1[nb][k];
  if constexpr (FE) {
    float* q2 = o.wpart + (size_t)blockIdx.x * 2 * H * H;
    float* q3 = q2 + H * H;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int jb = 0; jb < H / 16; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = n0 + nb * 16 + lg * 4 + r, n = jb * 16 + li;
          q2[m * H + n] = accW2[nb][jb][r];
          q3[m * H + n] = accW3[nb][jb][r];
        }
  }
}

// ---------------------------------------------------------------------------
#define XMGN_DISPATCH_T(prec, ...) \
  if (prec == 1) {                 \
    using T = bf16;                \
    __VA_ARGS__                    \
  } else {                         \
    using T = float;               \
    __VA_ARGS__                    \
  }
#define XMGN_DISPATCH_H(Hv, ...)                \
  if (Hv == 128) {                              \
    constexpr int H = 128;                      \
    __VA_ARGS__                                 \
  } else if (Hv == 256) {                       \
    constexpr int H = 256;                      \
    __VA_ARGS__                                 \
  } else if constexpr (sizeof(T) == 2) {        \
    constexpr int H = 512; /* BF16 only */      \
    __VA_ARGS__                                 \
  } else {                                      \
    g_config_error = 1;                         \
  }
#define XMGN_DISPATCH_ACT(a, ...) \
  if (a == 0) {                   \
    constexpr int ACT = 0;        \
    __VA_ARGS__                   \
  } else {                        \
    constexpr int ACT = 1;        \
    __VA_ARGS__                   \
  }
// Rows per tile: 64 or 32 at H = 128, 32 at H = 256 (LDS budget); at
// H = 512, 32 for edge tiles (whole receiver segments) and 16 for node tiles.
#define XMGN_DISPATCH_MT(mt, ...)          \
  if (mt == 64 && H == 128) {              \
    constexpr int MT = H == 128 ? 64 : 32; \
    __VA_ARGS__                            \
  } else if (mt == 16 && H == 512) {       \
    constexpr int MT = H == 512 ? 16 : 32; \
    __VA_ARGS__                            \
  } else {                                 \
    constexpr int MT = 32;                 \
    __VA_ARGS__                            \
  }
// Edge tiles (whole receiver segments): 64 or 32 rows at H = 128, and in the
// BF16 form also at H = 256 (a 64-row BF16 tile of [h_r | h_s | e] fits in
// LDS there and halves the weight bytes streamed per edge); 32 otherwise.
#define XMGN_DISPATCH_MT_EDGE(mt, ...)                                 \
  if (mt == 64 && (H == 128 || (H == 256 && sizeof(T) == 2))) {       \
    constexpr int MT = (H == 128 || (H == 256 && sizeof(T) == 2)) ? 64 : 32; \
    __VA_ARGS__                                                        \
  } else {                                                             \
    constexpr int MT = 32;                                             \
    __VA_ARGS__                                                        \
  }

template <typename T, int H, int MT>
constexpr bool edge_bwd_fits() {
  return (size_t)MT * (3 * H + 16 / sizeof(T)) * sizeof(T) + (size_t)MT * (H + 16 / sizeof(T)) * sizeof(T) +
             (size_t)MT * 4 * 8 <= 160 * 1024;
}
template <typename T, int H, int MT>
constexpr bool node_fits() {
  return 3 * (size_t)MT * (H + 16 / sizeof(T)) * sizeof(T) + (size_t)MT * (H + 4) * 4 + MT * 64 <= 160 * 1024 &&
         (size_t)MT * (2 * H + 16 / sizeof(T)) * sizeof(T) + (size_t)MT * (H + 4) * 4 <= 160 * 1024;
}

bool edge_bwd_fuses_wgrad(const Shape& s) { return s.prec == 1 && s.H == 128; }
bool edge_bwd_fuses_dw1e(const Shape& s, bool ztape) {
  return edge_bwd_fuses_wgrad(s) && !(ztape && s.mt_edge == 32);
}

template <int NW>
static void edge_bwd_nw(const Shape& s, const BatchView& b, const MlpW& w, const void* h, const void* e,
                        const void* zt, const void* at, const float* de_in, const float* dm, const EdgeBwdOut& o,
                        hipStream_t st) {
  XMGN_DISPATCH_T(s.prec, XMGN_DISPATCH_H(s.H, XMGN_DISPATCH_ACT(s.act, XMGN_DISPATCH_MT_EDGE(s.mt_edge, {
    // z from the tape: dW2-only fusion on 32-row tiles (two workgroups per
    // CU), both blocks fused on 64-row tiles; recompute: both fused
    constexpr int FW = (sizeof(T) == 2 && H == 128) ? (MT == 32 ? 2 : 1) : 0;
    constexpr int FWR = (sizeof(T) == 2 && H == 128) ? 1 : 0;
    constexpr int ZT = 1;
    if constexpr (edge_bwd_fits<T, H, MT>()) {
      if (zt && ACT != 0 && !at) {
        g_config_error = 1;
      } else if (zt) {
        if (s.agg)
          k_edge_bwd<T, H, MT, ACT, 1, FW, NW, ZT><<<s.grid, 64 * NW, 0, st>>>(
              b, w, (const T*)h, (const T*)e, (const T*)zt, (const T*)at, de_in, dm, o, s.eps);
        else
          k_edge_bwd<T, H, MT, ACT, 0, FW, NW, ZT><<<s.grid, 64 * NW, 0, st>>>(
              b, w, (const T*)h, (const T*)e, (const T*)zt, (const T*)at, de_in, dm, o, s.eps);
      } else {
        if (s.agg)
          k_edge_bwd<T, H, MT, ACT, 1, FWR, NW, 0><<<s.grid, 64 * NW, 0, st>>>(b, w, (const T*)h, (const T*)e, nullptr,
                                                                              nullptr, de_in, dm, o, s.eps);
        else
          k_edge_bwd<T, H, MT, ACT, 0, FWR, NW, 0><<<s.grid, 64 * NW, 0, st>>>(b, w, (const T*)h, (const T*)e, nullptr,
                                                                              nullptr, de_in, dm, o, s.eps);
      }
    } else {
      g_config_error = 1;
    }
  }))));
}

bool edge_z_tape(const Shape&) { return true; }
bool edge_a_tape(const Shape& s) { return s.act != 0; }

void launch_edge_bwd(const Shape& s, const BatchView& b, const MlpW& w, const void* h, const void* e,
                     const void* zt, const void* at, const float* de_in, const float* dm, const EdgeBwdOut& o,
                     hipStream_t st) {
  if (s.nw_edge == 8)
    edge_bwd_nw<8>(s, b, w, h, e, zt, at, de_in, dm, o, st);
  else
    edge_bwd_nw<4>(s, b, w, h, e, zt, at, de_in, dm, o, st);
}

void launch_node_bwd(const Shape& s, const BatchView& b, const MlpW& w, const void* h, const float* m,
                     const float* dh_in, const NodeBwdOut& o, hipStream_t st) {
  XMGN_DISPATCH_T(s.prec, XMGN_DISPATCH_H(s.H, XMGN_DISPATCH_ACT(s.act, XMGN_DISPATCH_MT(s.mt_node, {
    if constexpr (node_fits<T, H, MT>())
      k_node_bwd<T, H, MT, ACT><<<s.grid, NTHR, 0, st>>>(b.n, w, (const T*)h, m, dh_in, o, s.eps);
    else
      g_config_error = 1;
  }))));
}

void launch_node_dh(const Shape& s, const BatchView& b, const MlpW& w, const float* dh_mid, const float* S_r,
                    const float* S_s, float* dh_out, hipStream_t st) {
  XMGN_DISPATCH_T(s.prec, XMGN_DISPATCH_H(s.H, XMGN_DISPATCH_MT(s.mt_node, {
    if constexpr (node_fits<T, H, MT>())
      k_node_dh<T, H, MT><<<s.grid, NTHR, 0, st>>>(b.n, (const T*)w.Brs, dh_mid, S_r, S_s, dh_out);
    else
      g_config_error = 1;
  })));
}

void launch_sender_sum(const Shape& s, const BatchView& b, const void* da, float* S_s, hipStream_t st) {
  XMGN_DISPATCH_T(s.prec, XMGN_DISPATCH_H(s.H, {
    k_sender_sum<T, H><<<s.grid, NTHR, 0, st>>>(b.n, b.csc_ptr, b.csc_edge, (const T*)da, S_s);
  }));
}

void launch_dec_bwd(const Shape& s, const BatchView& b, const MlpW& w, const void* h, const float* d_out,
                    int out_dim, const DecBwdOut& o, hipStream_t st) {
  XMGN_DISPATCH_T(s.prec, XMGN_DISPATCH_H(s.H, XMGN_DISPATCH_ACT(s.act, XMGN_DISPATCH_MT(s.mt_node, {
    if constexpr (node_fits<T, H, MT>())
      k_dec_bwd<T, H, MT, ACT><<<s.grid, NTHR, 0, st>>>(b, w, (const T*)h, d_out, out_dim, o);
    else
      g_config_error = 1;
  }))));
}

void launch_enc_node_bwd(const Shape& s, const BatchView& b, const MlpW& w, const float* node_in, int in_dim,
                         const float* dh0, const EncBwdOut& o, hipStream_t st) {
  XMGN_DISPATCH_T(s.prec, XMGN_DISPATCH_H(s.H, XMGN_DISPATCH_ACT(s.act, XMGN_DISPATCH_MT(s.mt_node, {
    if constexpr (node_fits<T, H, MT>()) {
      if (in_dim <= 8)
        k_enc_bwd<T, H, MT, ACT, 0, 8><<<s.grid, NTHR, 0, st>>>(b.n, b, w, node_in, in_dim, dh0, o, s.eps);
      else if (o.da1)
        k_enc_bwd<T, H, MT, ACT, 0, 32><<<s.grid, NTHR, 0, st>>>(b.n, b, w, node_in, in_dim, dh0, o, s.eps);
      else
        g_config_error = 1;
    } else {
      g_config_error = 1;
    }
  }))));
}

void launch_enc_edge_bwd(const Shape& s, const BatchView& b, const MlpW& w, const float* xe, const float* de0,
                         const EncBwdOut& o, hipStream_t st) {
  XMGN_DISPATCH_T(s.prec, XMGN_DISPATCH_H(s.H, XMGN_DISPATCH_ACT(s.act, XMGN_DISPATCH_MT(enc_edge_rows(s), {
    if constexpr (node_fits<T, H, MT>())
      k_enc_bwd<T, H, MT, ACT, 1, 8><<<s.grid, NTHR, 0, st>>>(b.E, b, w, xe, 4, de0, o, s.eps);
    else
      g_config_error = 1;
  }))));
}

}  // namespace xmgn
