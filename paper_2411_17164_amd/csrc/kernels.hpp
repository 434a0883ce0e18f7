// Kernel argument blocks and launcher declarations of the xmgn library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xmgn {

// Set by a launcher when the requested tile configuration does not fit the
// hardware (LDS); the host turns it into XMGN_ERR_UNSUPPORTED.
extern int g_config_error;

// Device view of a batch (disjoint union of partitions).
struct BatchView {
  int n;                 // nodes
  int E;                 // edges
  const int* gid;        // [n] global node id
  const int* row_ptr;    // [n+1] receiver CSR
  const int* col;        // [E] sender (batch index)
  const int* recv;       // [E] receiver (batch index)
  const int* csc_ptr;    // [n+1] sender CSR
  const int* csc_edge;   // [E] CSR edge of each sender slot
  const int* etiles;     // [n_etiles+1][2] (receiver, edge) bounds of edge tiles
  int n_etiles;
  const int* inner;      // [n_inner] batch rows of inner nodes
  int n_inner;
};

// Per-MLP weight views.  W* are the compute-type copies ([out][in]);
// W*T are transposes ([in][out]) used by the backward products; vectors are
// FP32 views into the parameter blob.
struct MlpW {
  const void* W1;
  const void* W2;
  const void* W3;
  const void* W1T;  // edge: [H][H] block of W1^T for the e input; node/dec: full W1^T
  const void* W2T;
  const void* W3T;
  const void* Brs;  // edge layers: [H][2H] = [W1_r^T | W1_s^T]
  const float* W1f; // FP32 first-layer weights (encoders) / last layer (decoder)
  const float* b1;
  const float* b2;
  const float* b3;
  const float* gamma;
  const float* beta;
};

struct Shape {
  int H;
  int prec;     // 0 fp32, 1 bf16
  int act;      // 0 relu, 1 silu
  int agg;      // 0 message, 1 edge
  int mt_edge;  // rows per edge tile
  int mt_edge_bwd;  // rows per edge tile of the edge adjoint (its own tiling of the same edges)
  int mt_node;  // rows per node tile
  int grid;     // persistent grid (workgroups)
  int nw_edge;  // waves per workgroup of the edge kernels (4 or 8)
  int nw_edge_bwd;  // waves per workgroup of the edge adjoint
  float eps;
};

struct EdgeNorm {
  float mu[4];
  float sd[4];
};

// ---- forward ----
void launch_enc_node_fwd(const Shape& s, const BatchView& b, const MlpW& w, const float* node_in,
                         int in_dim, void* h0, hipStream_t st);
// Edge features ([x_s - x_r, |x_s - x_r|] - mu) / sd into xe[E][4].
void launch_edge_feat(const BatchView& b, const float* pos, EdgeNorm en, float* xe, hipStream_t st);
void launch_enc_edge_fwd(const Shape& s, const BatchView& b, const MlpW& w, const float* xe, void* e0,
                         hipStream_t st);
// z_out (or NULL): the hidden activation of every edge, for edge_z_tape forms;
// a_out (or NULL): its pre-activation, for edge_a_tape forms.
// pr, ps (or NULL for the gathered form): the node projections of
// launch_node_proj for this layer's edge MLP.
void launch_edge_fwd(const Shape& s, const BatchView& b, const MlpW& w, const void* h,
                     const void* e, void* e_out, float* m, void* z_out, void* a_out, const float* pr,
                     const float* ps, hipStream_t st);
// pr = W1_r h + b1, ps = W1_s h for every node (FP32 [n][H] each).
void launch_node_proj(const Shape& s, const BatchView& b, const MlpW& w, const void* h, float* pr, float* ps,
                      hipStream_t st);
void launch_node_fwd(const Shape& s, const BatchView& b, const MlpW& w, const void* h,
                     const float* m, void* h_out, hipStream_t st);
void launch_dec_fwd(const Shape& s, const BatchView& b, const MlpW& w, const void* h, float* out,
                    int out_dim, hipStream_t st);

// ---- backward ----
struct EdgeBwdOut {
  float* de_out;   // [E][H]
  float* S_r;      // [n][H] receiver sums of da
  void* da;        // [E][H] T
  void* du;        // [E][H] T
  void* z;         // [E][H] T
  float* partial;  // [grid][4H]: db1, db2, dgamma, dbeta
  float* wpart;    // fused weight gradients [grid][2][H][H] (dW2, e-block of dW1) or NULL
};
// True when the edge adjoint accumulates dW2 and the e-block of dW1 itself
// (then du and z are not written and wpart must be given).
bool edge_bwd_fuses_wgrad(const Shape& s);
// True when it also accumulates the e-block of dW1 (else that block is a
// separate product over da and e); s.mt_edge is the adjoint's tile rows.
bool edge_bwd_fuses_dw1e(const Shape& s, bool ztape);
// Fixed-order sums over the rows of partial matrices use a two-stage
// reduction with caller scratch of reduce_tmp_floats(columns) floats.
size_t reduce_tmp_floats(int max_cols);
void launch_wgrad_reduce(const float* partial, int n_chunks, int M_valid, int N, float* dst, int ldd, int MN,
                         float* tmp, hipStream_t st);
// True when the edge adjoint can read z from the forward's tape instead of
// recomputing it (every form); zt is then that tape (else NULL: recompute),
// and the unfused form does not write o.z (its dW2 product reads the tape).
bool edge_z_tape(const Shape& s);
// True when the forms that read z from the tape also need a (SiLU); at is
// then the tape of pre-activations (else NULL).
bool edge_a_tape(const Shape& s);
void launch_edge_bwd(const Shape& s, const BatchView& b, const MlpW& w, const void* h, const void* e,
                     const void* zt, const void* at, const float* de_in, const float* dm, const EdgeBwdOut& o,
                     hipStream_t st);

struct NodeBwdOut {
  float* dh_mid;   // [n][H]
  float* dm;       // [n][H]
  void* da;        // [n][H] T
  void* du;        // [n][H] T
  void* z;         // [n][H] T
  float* partial;  // [grid][4H]
  float* wpart;    // fused dW2 partials [grid][H][H] (or NULL)
};
// True when the node adjoint accumulates dW2 itself (then z and du are not
// written and wpart must be given); da is always written.
bool node_bwd_fuses_wgrad(const Shape& s);
void launch_node_bwd(const Shape& s, const BatchView& b, const MlpW& w, const void* h,
                     const float* m, const float* dh_in, const NodeBwdOut& o, hipStream_t st);
// dh_out = dh_mid + [S_r | S_s] * [W1_r ; W1_s]  (edge-layer input gradients)
void launch_node_dh(const Shape& s, const BatchView& b, const MlpW& w, const float* dh_mid,
                    const float* S_r, const float* S_s, float* dh_out, hipStream_t st);
void launch_sender_sum(const Shape& s, const BatchView& b, const void* da, float* S_s, hipStream_t st);

struct DecBwdOut {
  float* dh;       // [n][H], rows of inner nodes written (caller zeroes the rest)
  void* z1;        // [n_inner][H] T
  void* z2;
  void* da1;
  void* da2;
  float* dy;       // [n_inner][16]
  float* partial;  // [grid][2H + 16]
};
void launch_dec_bwd(const Shape& s, const BatchView& b, const MlpW& w, const void* h,
                    const float* d_out, int out_dim, const DecBwdOut& o, hipStream_t st);

struct EncBwdOut {
  void* z1;
  void* z2;
  void* da2;
  void* du3;
  float* partial;  // [grid][5H + 8H]: db1 db2 db3 dgamma dbeta dW1[H][8]
  float* wpart;    // fused weight gradients [grid][2][H][H] (dW2, dW3) or NULL
  float* da1;      // more than 8 inputs: adjoint of the input layer's output [rows][H] (FP32); dW1 not in partial
};
// Rows per tile of the edge encoder (no segment constraint): the edge tile
// at H = 128, the node tile at H = 256 and 512 (whose LDS budget it shares).
inline int enc_edge_rows(const Shape& s) { return s.H == 128 ? s.mt_edge : s.mt_node; }
// True when the encoder adjoint accumulates dW2 and dW3 itself (then z1,
// z2, da2 and du3 are not written and wpart must be given).
bool enc_bwd_fuses_wgrad(const Shape& s);
void launch_enc_node_bwd(const Shape& s, const BatchView& b, const MlpW& w, const float* node_in,
                         int in_dim, const float* dh0, const EncBwdOut& o, hipStream_t st);
void launch_enc_edge_bwd(const Shape& s, const BatchView& b, const MlpW& w, const float* xe, const float* de0,
                         const EncBwdOut& o, hipStream_t st);

// ---- auxiliary ----
// C[m][n] = sum_r A[ia(r)][a0 + m] * B[ib(r)][b0 + n] over r < R; partial
// sums per row chunk, then dst[m * ldd + n] = sum over chunks (m < M_valid).
struct WgradOp {
  const void* A;
  int a_f32;  // 1: A is FP32, else compute type
  int lda, a0;
  const int* ia;
  const void* B;
  int b_f32;
  int ldb, b0;
  const int* ib;
  int R, M, N, M_valid;
  float* dst;
  int ldd;
};
size_t wgrad_partial_floats(const Shape& s, const WgradOp& op);
void launch_wgrad(const Shape& s, const WgradOp& op, float* partial, float* tmp, hipStream_t st);

struct VecSeg {
  int src;  // offset in the partial row
  int len;
  float* dst;
};
// dst[j] = sum over g < G of partial[g * row + src + j] for every segment.
void launch_vec_reduce(const float* partial, int G, int row, const VecSeg* segs, int n_seg, float* tmp,
                       hipStream_t st);
void launch_vec_reduce_strided(const float* partial, int G, int row, int src, int runs, int inner, int src_stride,
                               float* dst, int dst_stride, float* tmp, hipStream_t st);

// A batch of the same fixed-order two-stage reductions, run as two launches
// in all: job j sets dst[m * ldd + n] = sum over r < rows of
// src[r * stride + m * N + n] (m < M_valid, n < N), with the split points
// and summation order of the single reductions above, so each result is
// bitwise the one a single reduction gives.
struct RedJob {
  const float* src;
  float* dst;
  int rows, stride, M_valid, N, ldd, splits, per;
  long long tmp_off;  // this job's stage-1 scratch, in floats
};
constexpr int kMaxRedJobs = 24;
struct RedBatch {
  int n = 0;
  int max_cols = 0;
  long long tmp_floats = 0;  // scratch the batch needs
  RedJob job[kMaxRedJobs];
  void add(const float* src, int rows, int stride, int M_valid, int N, float* dst, int ldd);
  // the segments of a per-workgroup partial row [G][row] (launch_vec_reduce)
  void add_vec(const float* partial, int G, int row, const VecSeg* segs, int n_seg);
};
void launch_reduce_batch(const RedBatch& b, float* tmp, hipStream_t st);
// The products of launch_wgrad without their reduction: adds that
// reduction to b.
void launch_wgrad_partials(const Shape& s, const WgradOp& op, float* partial, RedBatch& b, hipStream_t st);

struct PrepJob {
  int64_t src_off;   // element offset in the FP32 params
  int src_ld;        // row stride of the source matrix
  int src_col0;      // first source column
  int transpose;     // 0: dst[i][j] = src[i][col0 + j]; 1: dst[i][j] = src[j][col0 + i]
  int64_t dst_off;   // element offset in the compute blob
  int dst_ld;
  int dst_col0;
  int rows, cols;
};
void launch_prep(const float* params, void* blob, int prec, const PrepJob* jobs_dev, int n_jobs,
                 hipStream_t st);

void launch_fill(float* p, size_t n, float v, hipStream_t st);
void launch_accumulate(float* acc, const float* g, int64_t n, hipStream_t st);
// Adam constants of one step, each rounded to FP32 once from its FP64 value:
// c1 = 1 - b1, c2 = 1 - b2, bc1 = 1 - b1^t, bc2 = 1 - b2^t; clip <= 0: none.
struct AdamArgs {
  float lr, b1, b2, c1, c2, eps, bc1, bc2;
  double clip;
};
// partial: dev double [G] scratch; norm_out: dev float [1] or NULL.
void launch_adam(float* p, const float* g, float* m, float* v, int64_t n, double* partial, int G,
                 const AdamArgs& a, float* norm_out, hipStream_t st);
// Partials of the allocation-free optimizer step: the count launch_adam is
// given by both optimizer entry points, and the capacity of the library's
// fixed per-device array that the allocation-free one uses.
constexpr int kAdamScratchPartials = 256;
constexpr int kMaxDevices = 64;
// Device address (on `device`, which must be current) of that array; looked
// up on the first call per device.  Returns 0, or -1 (bad device) / -3
// (HIP error) with *err set.
int adam_noalloc_scratch(int device, double** out, const char** err);
void launch_mse(const float* out, const float* target, const int* gid, const int* inner, int n_inner,
                int out_dim, double inv_norm, float* d_out, float* partial, int G, float* loss,
                hipStream_t st);

// ---- kNN ----
int knn_build(const float* pos, int n, const int* level_end, int n_levels, int k_intra,
              int k_cross, int** row_ptr_out, int** col_out, long long* n_edges, hipStream_t st,
              const char** err);

}  // namespace xmgn
