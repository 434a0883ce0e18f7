// Forward kernels: node/edge encoders, the fused edge processor, the node
// processor and the decoder.  All are persistent-grid kernels over row tiles
// (see TileSched); each tile is staged in LDS, multiplied on MFMA with FP32
// accumulation, and post-processed (bias, activation, LayerNorm, residual)
// in registers before a coalesced write.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace xmgn {

template <typename T, int H, int NW = NWAVE>
struct Dims {
  static constexpr int PAD = 16 / sizeof(T);
  static constexpr int LDH = H + PAD;          // one H-wide tile
  static constexpr int LD2 = 2 * H + PAD;      // [h | m]
  static constexpr int LD3 = 3 * H + PAD;      // [h_r | h_s | e]
  static constexpr int LDF = H + 4;            // FP32 tile
  static constexpr int NB = H / (16 * NW);     // 16-column blocks per wave
  static constexpr int CPW = H / NW;           // columns per wave
};

// ---------------------------------------------------------------------------
// Fused edge processor, forward (Eq. 1-2):
//   x = [h_r ; h_s ; e],  v = LN(W2 act(W1 x + b1) + b2),  e' = e + v,
//   m_r = sum over the tile-local segment of r of v (or of e').
// A tile holds whole receiver segments, so m_r is summed in one workgroup in
// ascending sender order (the CSR order) -- deterministic, no atomics.
// ---------------------------------------------------------------------------
// NW waves per workgroup; each wave owns H / NW output columns of every GEMM.
// Gathered form: [h_s ; e] per edge (stride LD2) and h_r once per receiver
// of the tile (the tile's receivers are consecutive rows of h; MT rows at
// most), the first product reading each edge's h_r row through its
// receiver's tile-local index.
// SPLIT: the first layer's node blocks come precomputed per node (see
// k_node_proj), so only the e rows are gathered.  The FP32 tile of the
// segment sums aliases the staging tile; where it would be the larger (the
// split form), it holds one half of the columns at a time (NH = 2).
template <typename T, int H, int MT, int NW, int SPLIT = 0>
struct EdgeFwdLds {
  using D = Dims<T, H, NW>;
  static constexpr size_t ES = (size_t)MT * (SPLIT ? D::LDH : D::LD2) * sizeof(T);  // per-edge rows
  static constexpr size_t GS = ES + (SPLIT ? 0 : (size_t)MT * D::LDH * sizeof(T));  // + receiver rows
  static constexpr int NH = (size_t)MT * D::LDF * 4 > GS ? 2 : 1;
  static constexpr int LDFH = H / NH + 4;
  static constexpr size_t FS = (size_t)MT * LDFH * 4;
  static constexpr size_t XS = FS > GS ? FS : GS;
  static constexpr size_t ZS = (size_t)MT * D::LDH * sizeof(T);
  // receivers, senders, segment starts (MT + 1, padded)
  static constexpr size_t bytes = XS + ZS + 2 * NW * MT * 4 + (3 * MT + 4) * 4;
};

// z_out (or NULL): the hidden activation z = act(W1 x + b1) of every edge,
// kept for the adjoint; a_out (or NULL): its pre-activation a = W1 x + b1
// (SiLU's derivative needs a).
// SPLIT = 1: W1 x + b1 = W1_e e + (W1_r h_r + b1) + W1_s h_s, the last two
// read per edge from the FP32 node projections pr and ps (same value as the
// gathered form up to the rounding order of the sum).
template <typename T, int H, int MT, int ACT, int AGG, int NW, int SPLIT>
__global__ __launch_bounds__(64 * NW, waves_per_simd(EdgeFwdLds<T, H, MT, NW, SPLIT>::bytes, NW)) void k_edge_fwd(
    BatchView b, MlpW w, const T* __restrict__ h, const T* __restrict__ e, T* __restrict__ e_out,
    float* __restrict__ m, T* __restrict__ z_out, T* __restrict__ a_out, const float* __restrict__ pr,
    const float* __restrict__ ps, float eps) {
  using D = Dims<T, H, NW>;
  using L = EdgeFwdLds<T, H, MT, NW, SPLIT>;
  constexpr int LDX = SPLIT ? D::LDH : D::LD2;  // staging row stride
  constexpr int EC = SPLIT ? 0 : H;              // column of e in a staged row
  constexpr int MB = MT / 16, NB = D::NB;
  constexpr size_t XS = L::XS, ZS = L::ZS;
  constexpr int NH = L::NH, HH = H / NH, LDFH = L::LDFH;
  static_assert(NH == 1 || !SPLIT || D::CPW <= HH, "a wave's columns lie in one half");
  static_assert(SPLIT || NH == 1, "the gathered tile holds the whole FP32 tile");
  __shared__ __align__(16) unsigned char smem[L::bytes];
  T* xs = (T*)smem;
  T* hr = (T*)(smem + L::ES);  // gathered form: h_r of the tile's receivers
  float* ft = (float*)smem;  // aliases xs once the gathered tile is dead
  T* zs = (T*)(smem + XS);
  float* red = (float*)(smem + XS + ZS);
  int* rs = (int*)(red + 2 * NW * MT);
  int* ss = rs + MT;
  int* sg = rs + 2 * MT;
  const T* W1 = (const T*)w.W1;
  const T* W2 = (const T*)w.W2;
  const int n0 = wave_id() * D::CPW;

  TileSched sch(b.n_etiles);
  EdgeTilePipe ip;
  ip.start(b, sch);
  for (int t = sch.begin; t < sch.end; t += sch.step) {
    const EdgeTileIdx cur = ip.nx;
    const int r0 = cur.r0, r1 = cur.r1, e0 = cur.e0, ne = cur.ne;
    if (threadIdx.x < MT) {
      rs[threadIdx.x] = cur.rv;
      ss[threadIdx.x] = cur.cv;
    }
    lds_sync();
    if constexpr (!SPLIT) tile_segments(sg, rs, r0, r1, ne);  // read after the next barrier
    f32x4 acc[MB][NB];
    if constexpr (SPLIT) {
      gather_tile<T, D::LDH, MT, 1, H, 64 * NW>(
          xs, ne, [&](int, int i) { return e + (size_t)(e0 + i) * H; }, [](int, int, int, const uint4&) {});
      // the node blocks of the first product, in the accumulator layout:
      // acc = P_r[receiver] + P_s[sender], in flight during the barrier
      f32x4 sv[MB][NB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = acc_row(mb, r);
          const float* prow = pr + (size_t)rs[row] * H + n0 + (lane_id() & 15);
          const float* srow = ps + (size_t)ss[row] * H + n0 + (lane_id() & 15);
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            acc[mb][nb][r] = prow[16 * nb];
            sv[mb][nb][r] = srow[16 * nb];
          }
        }
      ip.advance(b, sch, t);  // next tile's indices and the bounds after, in flight from here
      lds_sync();
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[mb][nb][r] += sv[mb][nb][r];
      wave_gemm<T, MB, NB, H, D::LDH>(acc, xs, W1 + 2 * H, 3 * H, n0);  // + W1_e e
    } else {
      // one batch of loads: h_r of the nr receivers (consecutive rows of h),
      // then h_s and e of the ne edges
      const int nr = r1 - r0;
      constexpr int E8 = 16 / sizeof(T), CPR = H / E8, TOT = 3 * MT * CPR, IT = TOT / (64 * NW);
      static_assert(TOT % (64 * NW) == 0, "whole steps of the workgroup");
      uint4 v[IT];
#pragma unroll
      for (int k = 0; k < IT; ++k) {
        const int c = (int)threadIdx.x + k * 64 * NW, p = c / (MT * CPR), rem = c - p * (MT * CPR);
        const int i = rem / CPR, q = rem - i * CPR;
        const T* src = p == 0 ? h + (size_t)(r0 + i) * H : p == 1 ? h + (size_t)ss[i] * H : e + (size_t)(e0 + i) * H;
        v[k] = uint4{0u, 0u, 0u, 0u};
        if (i < (p == 0 ? nr : ne)) v[k] = *(const uint4*)(src + q * E8);
      }
#pragma unroll
      for (int k = 0; k < IT; ++k) {
        const int c = (int)threadIdx.x + k * 64 * NW, p = c / (MT * CPR), rem = c - p * (MT * CPR);
        const int i = rem / CPR, q = rem - i * CPR;
        *(uint4*)(p == 0 ? hr + i * D::LDH + q * E8 : xs + i * D::LD2 + (p - 1) * H + q * E8) = v[k];
      }
      ip.advance(b, sch, t);  // next tile's indices and the bounds after, in flight from here
      // each lane's h_r row (its row of every 16-row block): the receiver's tile-local index
      int roff[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int row = mb * 16 + (lane_id() & 15);
        roff[mb] = (row < ne ? rs[row] - r0 : 0) * D::LDH;
      }
      WFrag<T, NB, H> fr;
      fr.load(W1, 3 * H, n0);
      lds_sync();
      zero_acc(acc);
      wave_gemm_rows<T, MB, NB, H>(acc, hr, roff, fr);                // W1_r h_r
      wave_gemm<T, MB, NB, 2 * H, D::LD2>(acc, xs, W1 + H, 3 * H, n0);  // + W1_s h_s + W1_e e
    }
    f32x4 ev[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int c = acc_col(n0, nb);
        const float bb = SPLIT ? 0.f : w.b1[c];  // SPLIT: b1 is in P_r
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          acc[mb][nb][r] += bb;
          ev[mb][nb][r] = to_f(xs[acc_row(mb, r) * LDX + EC + c]);
        }
      }
    if (a_out) {  // uniform: the pre-activation goes out through zs first
      acc_to_lds<T, MB, NB, D::LDH>(acc, zs, n0);
      lds_sync();
      lds_rows_to_global<T, D::LDH>(zs, ne, H, a_out + (size_t)e0 * H, H, [](int i) { return i; });
      lds_sync();
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mb][nb][r] = act_f<ACT>(acc[mb][nb][r]);
    acc_to_lds<T, MB, NB, D::LDH>(acc, zs, n0);
    lds_sync();
    if (z_out) lds_rows_to_global<T, D::LDH>(zs, ne, H, z_out + (size_t)e0 * H, H, [](int i) { return i; });

    zero_acc(acc);
    wave_gemm<T, MB, NB, H, D::LDH>(acc, zs, W2, H, n0);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float bb = w.b2[acc_col(n0, nb)];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mb][nb][r] += bb;
      }
    float inv[MB][4];
    ln_normalize<MB, NB, MT, H, NW>(acc, red, eps, inv);  // barriers: GEMM2 done everywhere
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int c = acc_col(n0, nb);
        const float g = w.gamma[c], be = w.beta[c];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = acc_row(mb, r);
          const float v = g * acc[mb][nb][r] + be;
          const float en = ev[mb][nb][r] + v;
          acc[mb][nb][r] = AGG ? en : v;  // the summand of m
          zs[row * D::LDH + c] = from_f<T>(en);
        }
      }

    // m_r: sequential sum over the receiver's edges (ascending sender id),
    // NH column blocks of HH columns each
    const int nr = r1 - r0;
#pragma unroll
    for (int hf = 0; hf < NH; ++hf) {
      if (n0 / HH == hf)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) ft[acc_row(mb, r) * LDFH + acc_col(n0, nb) - hf * HH] = acc[mb][nb][r];
      lds_sync();
      for (int task = threadIdx.x; task < nr * (HH / 4); task += 64 * NW) {
        const int rl = task / (HH / 4), q = task - rl * (HH / 4);
        // (the split form reads the row pointers: the LDS starts cost it registers)
        const int lo = SPLIT ? b.row_ptr[r0 + rl] - e0 : sg[rl];
        const int hi = SPLIT ? b.row_ptr[r0 + rl + 1] - e0 : sg[rl + 1];
        float4 s = {0.f, 0.f, 0.f, 0.f};
        for (int i = lo; i < hi; ++i) {
          const float4 v = *(const float4*)(ft + i * LDFH + 4 * q);
          s.x += v.x;
          s.y += v.y;
          s.z += v.z;
          s.w += v.w;
        }
        *(float4*)(m + (size_t)(r0 + rl) * H + hf * HH + 4 * q) = s;
      }
      if (hf + 1 < NH) lds_sync();  // the next block overwrites the FP32 tile
    }
    if (e_out) lds_rows_to_global<T, D::LDH>(zs, ne, H, e_out + (size_t)e0 * H, H, [](int i) { return i; });
    lds_sync();
  }
}

// ---------------------------------------------------------------------------
// Wide edge forward (BF16 gathered form at H = 256 and 512): the same MLP as
// k_edge_fwd's gathered form, with the first product over K slices of 64
// columns of the gathered [h_r ; h_s ; e] rows, double-buffered in LDS: the
// next slice's rows and weight fragments are in flight while the current
// slice's MFMAs run.  Only a slice of the gathered tile is ever in LDS, so
// tiles can be taller than a whole gathered tile allows (64 rows at
// H = 512, where each weight element streamed from L2 then serves twice as
// many edges; 128 at H = 256), or, at the same height (64 rows, 4 waves, at
// H = 256), small enough for two workgroups per CU.  After the second
// product e is staged in the z tile's place; the FP32 segment-sum tile then
// takes that place, one half of the columns at a time.
// ---------------------------------------------------------------------------
template <int H, int MT, int NW_ = 8>
struct EdgeFwdWide {
  static constexpr int NW = NW_, NT = 64 * NW;
  static constexpr int KS = 64, LDK = KS + 8;         // slice width, slice row stride
  static constexpr int NS = 3 * H / KS;               // slices of [h_r ; h_s ; e]
  static constexpr int LDH = H + 8;
  static constexpr size_t SL = (size_t)MT * LDK * 2;  // one slice buffer
  static constexpr size_t ZS = (size_t)MT * LDH * 2;  // z, then e and e', then the FP32 tile
  static constexpr int FC = H / 2, LDF = FC + 4;      // FP32 tile: half of the columns
  static_assert((size_t)MT * LDF * 4 <= ZS, "FP32 half tile fits in the z tile");
  static constexpr size_t bytes = 2 * SL + ZS + 2 * NW * MT * 4 + 2 * MT * 4;
};

template <int H, int MT, int ACT, int AGG, int NWW>
__global__ __launch_bounds__(64 * NWW, (waves_per_simd(EdgeFwdWide<H, MT, NWW>::bytes, NWW))) void k_edge_fwd_wide(
    BatchView b, MlpW w, const bf16* __restrict__ h,
                                                         const bf16* __restrict__ e, bf16* __restrict__ e_out,
                                                         float* __restrict__ m, bf16* __restrict__ z_out,
                                                         bf16* __restrict__ a_out, float eps) {
  using L = EdgeFwdWide<H, MT, NWW>;
  constexpr int NW = L::NW, NT = L::NT, KS = L::KS, LDK = L::LDK, NS = L::NS, LDH = L::LDH;
  constexpr int FC = L::FC, LDF = L::LDF;
  constexpr int CPW = H / NW, NB = CPW / 16, MB = MT / 16;
  static_assert(NS % 2 == 0, "slices go in pairs");
  static_assert(CPW <= FC, "a wave's columns lie in one half");
  constexpr int CPRS = KS / 8, SLT = MT * CPRS, SIT = SLT / NT;  // 16-byte chunks of a slice
  static_assert(SLT % NT == 0, "whole steps of the workgroup");
  __shared__ __align__(16) unsigned char smem[L::bytes];
  bf16* sl0 = (bf16*)smem;
  bf16* sl1 = (bf16*)(smem + L::SL);
  bf16* zs = (bf16*)(smem + 2 * L::SL);
  float* ft = (float*)zs;
  float* red = (float*)(smem + 2 * L::SL + L::ZS);
  int* rs = (int*)(red + 2 * NW * MT);
  int* ss = rs + MT;
  const bf16* W1 = (const bf16*)w.W1;
  const bf16* W2 = (const bf16*)w.W2;
  const int n0 = wave_id() * CPW;

  TileSched sch(b.n_etiles);
  EdgeTilePipe ip;
  ip.start(b, sch);
  for (int t = sch.begin; t < sch.end; t += sch.step) {
    const EdgeTileIdx cur = ip.nx;
    const int r0 = cur.r0, r1 = cur.r1, e0 = cur.e0, ne = cur.ne;
    if (threadIdx.x < MT) {
      rs[threadIdx.x] = cur.rv;
      ss[threadIdx.x] = cur.cv;
    }
    lds_sync();
    uint4 v[SIT];
    auto load_slice = [&](int sl) {
      const int p = sl / (H / KS), c0 = (sl % (H / KS)) * KS;
#pragma unroll
      for (int k = 0; k < SIT; ++k) {
        const int c = (int)threadIdx.x + k * NT, i = c / CPRS, q = c - i * CPRS;
        v[k] = uint4{0u, 0u, 0u, 0u};
        if (i < ne) {
          const bf16* row = p == 0 ? h + (size_t)rs[i] * H : p == 1 ? h + (size_t)ss[i] * H : e + (size_t)(e0 + i) * H;
          v[k] = *(const uint4*)(row + c0 + q * 8);
        }
      }
    };
    auto store_slice = [&](bf16* buf) {
#pragma unroll
      for (int k = 0; k < SIT; ++k) {
        const int c = (int)threadIdx.x + k * NT, i = c / CPRS, q = c - i * CPRS;
        *(uint4*)(buf + i * LDK + q * 8) = v[k];
      }
    };
    f32x4 acc[MB][NB];
    zero_acc(acc);
    WFrag<bf16, NB, KS> fa, fb;
    load_slice(0);
    fa.load(W1, 3 * H, n0);
    store_slice(sl0);
    ip.advance(b, sch, t);  // next tile's indices and the bounds after, in flight from here
#pragma unroll 1
    for (int sl = 0; sl < NS; sl += 2) {
      // slice sl from sl0 with fa; slice sl + 1 and its weights in flight
      load_slice(sl + 1);
      fb.load(W1 + (sl + 1) * KS, 3 * H, n0);
      lds_sync();  // slice sl stored by every wave; slice sl - 1's products done with sl1
      wave_gemm<bf16, MB, NB, KS, LDK>(acc, sl0, fa);
      store_slice(sl1);
      // slice sl + 1 from sl1 with fb
      if (sl + 2 < NS) {
        load_slice(sl + 2);
        fa.load(W1 + (sl + 2) * KS, 3 * H, n0);
      }
      lds_sync();
      wave_gemm<bf16, MB, NB, KS, LDK>(acc, sl1, fb);
      if (sl + 2 < NS) store_slice(sl0);
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float bb = w.b1[acc_col(n0, nb)];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mb][nb][r] += bb;
      }
    if (a_out) {  // uniform: the pre-activation goes out through zs first
      acc_to_lds<bf16, MB, NB, LDH>(acc, zs, n0);
      lds_sync();
      lds_rows_to_global<bf16, LDH>(zs, ne, H, a_out + (size_t)e0 * H, H, [](int i) { return i; });
      lds_sync();
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mb][nb][r] = act_f<ACT>(acc[mb][nb][r]);
    acc_to_lds<bf16, MB, NB, LDH>(acc, zs, n0);
    lds_sync();
    if (z_out) lds_rows_to_global<bf16, LDH>(zs, ne, H, z_out + (size_t)e0 * H, H, [](int i) { return i; });
    zero_acc(acc);
    wave_gemm<bf16, MB, NB, H, LDH>(acc, zs, W2, H, n0);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float bb = w.b2[acc_col(n0, nb)];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mb][nb][r] += bb;
      }
    float inv[MB][4];
    ln_normalize<MB, NB, MT, H, NW>(acc, red, eps, inv);  // barriers: every wave is done with z
    // e of the tile's edges, in the z tile's place
    gather_tile<bf16, LDH, MT, 1, H, NT>(
        zs, ne, [&](int, int i) { return e + (size_t)(e0 + i) * H; }, [](int, int, int, const uint4&) {});
    lds_sync();
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int c = acc_col(n0, nb);
        const float g = w.gamma[c], be = w.beta[c];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = acc_row(mb, r);
          const float vv = g * acc[mb][nb][r] + be;
          const float en = to_f(zs[row * LDH + c]) + vv;
          acc[mb][nb][r] = AGG ? en : vv;  // the summand of m
          zs[row * LDH + c] = from_f<bf16>(en);
        }
      }
    lds_sync();
    if (e_out) lds_rows_to_global<bf16, LDH>(zs, ne, H, e_out + (size_t)e0 * H, H, [](int i) { return i; });
    lds_sync();  // e' is out: the FP32 tile takes its place
    // m_r: sequential sum over the receiver's edges (ascending sender id), one column half at a time
    const int nr = r1 - r0;
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      if (n0 / FC == hf)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) ft[acc_row(mb, r) * LDF + acc_col(n0, nb) - hf * FC] = acc[mb][nb][r];
      lds_sync();
      for (int task = threadIdx.x; task < nr * (FC / 4); task += NT) {
        const int rl = task / (FC / 4), q = task - rl * (FC / 4);
        const int lo = b.row_ptr[r0 + rl] - e0, hi = b.row_ptr[r0 + rl + 1] - e0;
        float4 sm = {0.f, 0.f, 0.f, 0.f};
        for (int i = lo; i < hi; ++i) {
          const float4 x = *(const float4*)(ft + i * LDF + 4 * q);
          sm.x += x.x;
          sm.y += x.y;
          sm.z += x.z;
          sm.w += x.w;
        }
        *(float4*)(m + (size_t)(r0 + rl) * H + hf * FC + 4 * q) = sm;
      }
      lds_sync();
    }
  }
}

// ---------------------------------------------------------------------------
// Node projections of the edge MLP's first layer (Eq. 1 re-associated): the
// blocks of W1 that act on the receiver's and the sender's latent give
//   pr = W1_r h + b1,  ps = W1_s h   (FP32, [n][H] each)
// once per node instead of once per edge; the edge forward's split form
// then needs only W1_e e per edge.
// ---------------------------------------------------------------------------
template <typename T, int H, int MT>
__global__ __launch_bounds__(NTHR, 2) void k_node_proj(int n, MlpW w, const T* __restrict__ h, float* __restrict__ pr,
                                                      float* __restrict__ ps) {
  using D = Dims<T, H>;
  constexpr int MB = MT / 16, NB = D::NB;
  constexpr size_t XS = (size_t)MT * D::LDH * sizeof(T);
  __shared__ __align__(16) unsigned char smem[XS + (size_t)MT * D::LDF * 4];
  T* xs = (T*)smem;
  float* ft = (float*)(smem + XS);
  const T* W1 = (const T*)w.W1;
  const int n0 = wave_id() * D::CPW;
  const int n_tiles = (n + MT - 1) / MT;
  TileSched sch(n_tiles);
  for (int t = sch.begin; t < sch.end; t += sch.step) {
    const int row0 = t * MT, nr = min(MT, n - row0);
    global_rows_to_lds<T, D::LDH, MT, H>(xs, nr, 0, [&](int i) { return h + (size_t)(row0 + i) * H; });
    lds_sync();
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      f32x4 acc[MB][NB];
      zero_acc(acc);
      wave_gemm<T, MB, NB, H, D::LDH>(acc, xs, W1 + blk * H, 3 * H, n0);
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const int c = acc_col(n0, nb);
          const float bb = blk == 0 ? w.b1[c] : 0.f;
#pragma unroll
          for (int r = 0; r < 4; ++r) ft[acc_row(mb, r) * D::LDF + c] = acc[mb][nb][r] + bb;
        }
      lds_sync();
      float* dst = blk == 0 ? pr : ps;
      for (int c = threadIdx.x; c < nr * (H / 4); c += NTHR) {
        const int i = c / (H / 4), q = c - i * (H / 4);
        *(float4*)(dst + (size_t)(row0 + i) * H + 4 * q) = *(const float4*)(ft + i * D::LDF + 4 * q);
      }
      lds_sync();
    }
  }
}

// ---------------------------------------------------------------------------
// Node processor, forward (Eq. 3): h' = h + LN(W2 act(W1 [h ; m] + b1) + b2)
// ---------------------------------------------------------------------------
template <typename T, int H, int MT, int ACT>
__global__ __launch_bounds__(NTHR, H == 128 ? 2 : 1) void k_node_fwd(int n, MlpW w, const T* __restrict__ h,
                                                   const float* __restrict__ m, T* __restrict__ h_out,
                                                   float eps) {
  using D = Dims<T, H>;
  constexpr int MB = MT / 16, NB = D::NB;
  constexpr size_t XS = (size_t)MT * D::LD2 * sizeof(T);
  constexpr size_t ZS = (size_t)MT * D::LDH * sizeof(T);
  __shared__ __align__(16) unsigned char smem[XS + ZS + 2 * NWAVE * MT * 4];
  T* xs = (T*)smem;
  T* zs = (T*)(smem + XS);
  float* red = (float*)(smem + XS + ZS);
  const T* W1 = (const T*)w.W1;
  const T* W2 = (const T*)w.W2;
  const int n0 = wave_id() * D::CPW;
  const int n_tiles = (n + MT - 1) / MT;

  // H = 128: the next tile's h and m rows travel in registers while this
  // tile computes, so their HBM round trip is off the tile's critical path
  // (wider forms have no registers to spare)
  constexpr bool PF = H == 128;
  TileSched sch(n_tiles);
  NodeRowsPre<T, H, MT, D::LD2> pre;
  if constexpr (PF)
    if (sch.begin < sch.end) pre.load(h, m, sch.begin * MT, min(MT, n - sch.begin * MT));
  for (int t = sch.begin; t < sch.end; t += sch.step) {
    const int row0 = t * MT, nr = min(MT, n - row0);
    if constexpr (PF) {
      pre.store(xs);
      if (t + sch.step < sch.end) pre.load(h, m, (t + sch.step) * MT, min(MT, n - (t + sch.step) * MT));
    } else {
      global_rows_to_lds<T, D::LD2, MT, H>(xs, nr, 0, [&](int i) { return h + (size_t)(row0 + i) * H; });
      global_f32_rows_to_lds<T, D::LD2, MT, H>(xs, nr, H, [&](int i) { return m + (size_t)(row0 + i) * H; });
    }
    lds_sync();
    f32x4 acc[MB][NB];
    zero_acc(acc);
    wave_gemm<T, MB, NB, 2 * H, D::LD2>(acc, xs, W1, 2 * H, n0);
    f32x4 hv[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int c = acc_col(n0, nb);
        const float bb = w.b1[c];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          acc[mb][nb][r] = act_f<ACT>(acc[mb][nb][r] + bb);
          hv[mb][nb][r] = to_f(xs[acc_row(mb, r) * D::LD2 + c]);
        }
      }
    acc_to_lds<T, MB, NB, D::LDH>(acc, zs, n0);
    lds_sync();
    zero_acc(acc);
    wave_gemm<T, MB, NB, H, D::LDH>(acc, zs, W2, H, n0);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float bb = w.b2[acc_col(n0, nb)];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mb][nb][r] += bb;
      }
    float inv[MB][4];
    ln_normalize<MB, NB, MT, H>(acc, red, eps, inv);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int c = acc_col(n0, nb);
        const float g = w.gamma[c], be = w.beta[c];
#pragma unroll
        for (int r = 0; r < 4; ++r)
          zs[acc_row(mb, r) * D::LDH + c] = from_f<T>(hv[mb][nb][r] + g * acc[mb][nb][r] + be);
      }
    lds_sync();
    lds_rows_to_global<T, D::LDH>(zs, nr, H, h_out + (size_t)row0 * H, H, [](int i) { return i; });
    lds_sync();
  }
}

// ---------------------------------------------------------------------------
// Encoders: in -> H -> H -> H, LN.  The first layer (in <= 8) is a plain FMA
// product in the accumulator layout; the other two run on MFMA.
// Node input: node_in[gid]; edge input: the edge features of k_edge_feat.
// ---------------------------------------------------------------------------
// Edge features ([x_s - x_r, |x_s - x_r|] - mu) / sd, one float4 per edge
// (Sec. III.B), computed once per forward and read by both edge encoders.
__global__ __launch_bounds__(256) void k_edge_feat(int E, BatchView b, const float* __restrict__ pos, EdgeNorm en,
                                                   float4* __restrict__ xe) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= E) return;
  const float* ps = pos + (size_t)b.gid[b.col[k]] * 3;
  const float* pr = pos + (size_t)b.gid[b.recv[k]] * 3;
  const float dx = ps[0] - pr[0], dy = ps[1] - pr[1], dz = ps[2] - pr[2];
  const float d = sqrtf(dx * dx + dy * dy + dz * dz);
  xe[k] = float4{(dx - en.mu[0]) / en.sd[0], (dy - en.mu[1]) / en.sd[1], (dz - en.mu[2]) / en.sd[2],
                 (d - en.mu[3]) / en.sd[3]};
}

void launch_edge_feat(const BatchView& b, const float* pos, EdgeNorm en, float* xe, hipStream_t st) {
  if (b.E == 0) return;
  k_edge_feat<<<(b.E + 255) / 256, 256, 0, st>>>(b.E, b, pos, en, (float4*)xe);
}

// KIN: input slots per row (8, or 32 for up to 32 inputs, whose first layer
// reads its weights from global memory inside a runtime-length loop).
template <typename T, int H, int MT, int ACT, int KIND, int KIN>
__global__ __launch_bounds__(NTHR, H == 128 ? 2 : 1) void k_enc_fwd(int rows, BatchView b, MlpW w, const float* __restrict__ src,
                                                  int in_dim, T* __restrict__ out, float eps) {
  using D = Dims<T, H>;
  constexpr int MB = MT / 16, NB = D::NB;
  constexpr size_t ZS = (size_t)MT * D::LDH * sizeof(T);
  __shared__ __align__(16) unsigned char smem[2 * ZS + MT * KIN * 4 + 2 * NWAVE * MT * 4];
  T* zs = (T*)smem;
  T* z2 = (T*)(smem + ZS);
  float* xin = (float*)(smem + 2 * ZS);
  float* red = xin + MT * KIN;  // [2][NWAVE][MT]
  const T* W2 = (const T*)w.W2;
  const T* W3 = (const T*)w.W3;
  const int n0 = wave_id() * D::CPW;
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
    f32x4 acc[MB][NB];
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
            const float* x = xin + acc_row(mb, r) * 8;
            float a = bb;
#pragma unroll
            for (int k = 0; k < 8; ++k) a += wr[k] * x[k];
            acc[mb][nb][r] = act_f<ACT>(a);
          }
      } else {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[mb][nb][r] = bb;
        for (int k = 0; k < in_dim; ++k) {
          const float wk = w.W1f[c * in_dim + k];
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[mb][nb][r] += wk * xin[acc_row(mb, r) * KIN + k];
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[mb][nb][r] = act_f<ACT>(acc[mb][nb][r]);
      }
    }
    acc_to_lds<T, MB, NB, D::LDH>(acc, zs, n0);
    lds_sync();
    zero_acc(acc);
    wave_gemm<T, MB, NB, H, D::LDH>(acc, zs, W2, H, n0);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float bb = w.b2[acc_col(n0, nb)];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mb][nb][r] = act_f<ACT>(acc[mb][nb][r] + bb);
      }
    acc_to_lds<T, MB, NB, D::LDH>(acc, z2, n0);
    lds_sync();
    zero_acc(acc);
    wave_gemm<T, MB, NB, H, D::LDH>(acc, z2, W3, H, n0);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float bb = w.b3[acc_col(n0, nb)];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mb][nb][r] += bb;
      }
    float inv[MB][4];
    ln_normalize<MB, NB, MT, H>(acc, red, eps, inv);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int c = acc_col(n0, nb);
        const float g = w.gamma[c], be = w.beta[c];
#pragma unroll
        for (int r = 0; r < 4; ++r) zs[acc_row(mb, r) * D::LDH + c] = from_f<T>(g * acc[mb][nb][r] + be);
      }
    lds_sync();
    lds_rows_to_global<T, D::LDH>(zs, nr, H, out + (size_t)row0 * H, H, [](int i) { return i; });
    lds_sync();
  }
}

// ---------------------------------------------------------------------------
// Decoder: y = W3 act(W2 act(W1 h + b1) + b2) + b3 on the batch's inner rows,
// written to out[gid][0:out_dim].  The last layer (out_dim <= 16) is FMA.
// ---------------------------------------------------------------------------
template <typename T, int H, int MT, int ACT>
__global__ __launch_bounds__(NTHR, H == 128 ? 2 : 1) void k_dec_fwd(BatchView b, MlpW w, const T* __restrict__ h,
                                                  float* __restrict__ out, int out_dim) {
  using D = Dims<T, H>;
  constexpr int MB = MT / 16, NB = D::NB;
  constexpr size_t ZS = (size_t)MT * D::LDH * sizeof(T);
  __shared__ __align__(16) unsigned char smem[2 * ZS];
  T* xs = (T*)smem;
  T* zs = (T*)(smem + ZS);
  const T* W1 = (const T*)w.W1;
  const T* W2 = (const T*)w.W2;
  const int n0 = wave_id() * D::CPW;
  const int n_tiles = (b.n_inner + MT - 1) / MT;

  TileSched sch(n_tiles);
  for (int t = sch.begin; t < sch.end; t += sch.step) {
    const int row0 = t * MT, nr = min(MT, b.n_inner - row0);
    global_rows_to_lds<T, D::LDH, MT, H>(xs, nr, 0, [&](int i) { return h + (size_t)b.inner[row0 + i] * H; });
    lds_sync();
    f32x4 acc[MB][NB];
    zero_acc(acc);
    wave_gemm<T, MB, NB, H, D::LDH>(acc, xs, W1, H, n0);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float bb = w.b1[acc_col(n0, nb)];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mb][nb][r] = act_f<ACT>(acc[mb][nb][r] + bb);
      }
    acc_to_lds<T, MB, NB, D::LDH>(acc, zs, n0);
    lds_sync();
    zero_acc(acc);
    wave_gemm<T, MB, NB, H, D::LDH>(acc, zs, W2, H, n0);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float bb = w.b2[acc_col(n0, nb)];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mb][nb][r] = act_f<ACT>(acc[mb][nb][r] + bb);
      }
    acc_to_lds<T, MB, NB, D::LDH>(acc, xs, n0);
    lds_sync();
    for (int task = threadIdx.x; task < nr * out_dim; task += NTHR) {
      const int i = task / out_dim, o = task - i * out_dim;
      const float* wr = w.W1f + (size_t)o * H;  // decoder W3 (FP32)
      const T* z = xs + i * D::LDH;
      float y = 0.f;
      for (int j = 0; j < H; ++j) y += wr[j] * to_f(z[j]);
      out[(size_t)b.gid[b.inner[row0 + i]] * out_dim + o] = y + w.b3[o];
    }
    lds_sync();
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define XMGN_DISPATCH_T(prec, ...)      \
  if (prec == 1) {                      \
    using T = bf16;                     \
    __VA_ARGS__                         \
  } else {                              \
    using T = float;                    \
    __VA_ARGS__                         \
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
#define XMGN_DISPATCH_ACT(a, ...)       \
  if (a == 0) {                         \
    constexpr int ACT = 0;              \
    __VA_ARGS__                         \
  } else {                              \
    constexpr int ACT = 1;              \
    __VA_ARGS__                         \
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
constexpr bool edge_fits() {
  return (size_t)MT * (3 * H + 16 / sizeof(T)) * sizeof(T) + (size_t)MT * (H + 16 / sizeof(T)) * sizeof(T) +
             (size_t)MT * 4 * 8 <= 160 * 1024;
}

template <int NW>
static void edge_fwd_nw(const Shape& s, const BatchView& b, const MlpW& w, const void* h, const void* e, void* e_out,
                        float* m, void* z_out, void* a_out, const float* pr, const float* ps, hipStream_t st) {
  XMGN_DISPATCH_T(s.prec, XMGN_DISPATCH_H(s.H, XMGN_DISPATCH_ACT(s.act, XMGN_DISPATCH_MT_EDGE(s.mt_edge, {
    if constexpr (edge_fits<T, H, MT>()) {
      auto go = [&](auto agg, auto split) {
        k_edge_fwd<T, H, MT, ACT, decltype(agg)::value, NW, decltype(split)::value><<<s.grid, 64 * NW, 0, st>>>(
            b, w, (const T*)h, (const T*)e, (T*)e_out, m, (T*)z_out, (T*)a_out, pr, ps, s.eps);
      };
      using I0 = std::integral_constant<int, 0>;
      using I1 = std::integral_constant<int, 1>;
      if (pr) {
        if (s.agg) go(I1{}, I1{}); else go(I0{}, I1{});
      } else {
        if (s.agg) go(I1{}, I0{}); else go(I0{}, I0{});
      }
    } else {
      g_config_error = 1;
    }
  }))));
}

// The BF16 gathered form at H = 256 (64- and 128-row tiles) and at H = 512
// (64-row tiles) runs the wide kernel.
bool edge_fwd_wide(const Shape& s) {
  return s.prec == 1 && ((s.H == 256 && (s.mt_edge == 128 || s.mt_edge == 64)) || (s.H == 512 && s.mt_edge == 64));
}

void launch_edge_fwd(const Shape& s, const BatchView& b, const MlpW& w, const void* h, const void* e,
                     void* e_out, float* m, void* z_out, void* a_out, const float* pr, const float* ps,
                     hipStream_t st) {
  if (b.n_etiles == 0) return;
  if (edge_fwd_wide(s) && !pr) {  // the split form runs k_edge_fwd (128-row tiles never reach it)
    auto go = [&](auto hh, auto mt, auto act, auto agg) {
      constexpr int NWW = decltype(hh)::value == 256 && decltype(mt)::value == 64 ? 4 : 8;
      k_edge_fwd_wide<decltype(hh)::value, decltype(mt)::value, decltype(act)::value, decltype(agg)::value, NWW>
          <<<s.grid, 64 * NWW, 0, st>>>(b, w, (const bf16*)h, (const bf16*)e, (bf16*)e_out, m, (bf16*)z_out,
                                        (bf16*)a_out, s.eps);
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    auto by_h = [&](auto act, auto agg) {
      if (s.H == 256 && s.mt_edge == 128)
        go(std::integral_constant<int, 256>{}, std::integral_constant<int, 128>{}, act, agg);
      else if (s.H == 256)
        go(std::integral_constant<int, 256>{}, std::integral_constant<int, 64>{}, act, agg);
      else
        go(std::integral_constant<int, 512>{}, std::integral_constant<int, 64>{}, act, agg);
    };
    if (s.act) {
      if (s.agg) by_h(I1{}, I1{}); else by_h(I1{}, I0{});
    } else {
      if (s.agg) by_h(I0{}, I1{}); else by_h(I0{}, I0{});
    }
    return;
  }
  if (s.nw_edge == 8)
    edge_fwd_nw<8>(s, b, w, h, e, e_out, m, z_out, a_out, pr, ps, st);
  else
    edge_fwd_nw<4>(s, b, w, h, e, e_out, m, z_out, a_out, pr, ps, st);
}

void launch_node_proj(const Shape& s, const BatchView& b, const MlpW& w, const void* h, float* pr, float* ps,
                      hipStream_t st) {
  if (b.n == 0) return;
  XMGN_DISPATCH_T(s.prec, XMGN_DISPATCH_H(s.H, {
    constexpr int MT = H == 512 ? 16 : 32;
    k_node_proj<T, H, MT><<<s.grid, NTHR, 0, st>>>(b.n, w, (const T*)h, pr, ps);
  }));
}

void launch_node_fwd(const Shape& s, const BatchView& b, const MlpW& w, const void* h, const float* m,
                     void* h_out, hipStream_t st) {
  if (b.n == 0) return;
  XMGN_DISPATCH_T(s.prec, XMGN_DISPATCH_H(s.H, XMGN_DISPATCH_ACT(s.act, XMGN_DISPATCH_MT(s.mt_node, {
    k_node_fwd<T, H, MT, ACT><<<s.grid, NTHR, 0, st>>>(b.n, w, (const T*)h, m, (T*)h_out, s.eps);
  }))));
}

void launch_enc_node_fwd(const Shape& s, const BatchView& b, const MlpW& w, const float* node_in, int in_dim,
                         void* h0, hipStream_t st) {
  if (b.n == 0) return;
  XMGN_DISPATCH_T(s.prec, XMGN_DISPATCH_H(s.H, XMGN_DISPATCH_ACT(s.act, XMGN_DISPATCH_MT(s.mt_node, {
    if (in_dim <= 8)
      k_enc_fwd<T, H, MT, ACT, 0, 8><<<s.grid, NTHR, 0, st>>>(b.n, b, w, node_in, in_dim, (T*)h0, s.eps);
    else
      k_enc_fwd<T, H, MT, ACT, 0, 32><<<s.grid, NTHR, 0, st>>>(b.n, b, w, node_in, in_dim, (T*)h0, s.eps);
  }))));
}

void launch_enc_edge_fwd(const Shape& s, const BatchView& b, const MlpW& w, const float* xe, void* e0,
                         hipStream_t st) {
  if (b.E == 0) return;
  XMGN_DISPATCH_T(s.prec, XMGN_DISPATCH_H(s.H, XMGN_DISPATCH_ACT(s.act, XMGN_DISPATCH_MT(enc_edge_rows(s), {
    k_enc_fwd<T, H, MT, ACT, 1, 8><<<s.grid, NTHR, 0, st>>>(b.E, b, w, xe, 4, (T*)e0, s.eps);
  }))));
}

void launch_dec_fwd(const Shape& s, const BatchView& b, const MlpW& w, const void* h, float* out, int out_dim,
                    hipStream_t st) {
  if (b.n_inner == 0) return;
  XMGN_DISPATCH_T(s.prec, XMGN_DISPATCH_H(s.H, XMGN_DISPATCH_ACT(s.act, XMGN_DISPATCH_MT(s.mt_node, {
    k_dec_fwd<T, H, MT, ACT><<<s.grid, NTHR, 0, st>>>(b, w, (const T*)h, out, out_dim);
  }))));
}

}  // namespace xmgn
