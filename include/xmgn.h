/*
 * xmgn.h -- C ABI of the MI355X (gfx950) X-MeshGraphNet processor library.
 *
 * The library builds multi-scale kNN graphs from point clouds, splits them
 * into partitions with an L-hop halo, and runs the MeshGraphNet
 * encoder / processor / decoder forward and its hand-written adjoint over a
 * batch of partitions on one GPU, with gradients aggregated over partitions.
 *
 * Conventions (every call):
 *  - Return XMGN_OK (0) or a negative XMGN_ERR_* code; xmgn_last_error()
 *    then describes the failure.  No C++ exception crosses this boundary.
 *  - "dev" pointers are HIP device memory, "host" pointers host memory.  All
 *    arrays are dense and row-major.  The caller owns every buffer it passes;
 *    the library never frees or keeps a caller pointer beyond the call.
 *  - Handles (xmgn_ctx, xmgn_graph, xmgn_partset) are owned by the library and
 *    released with the matching *_destroy call.
 *  - Device work is enqueued asynchronously on the given stream (a
 *    hipStream_t; NULL = the null stream).  Only xmgn_build_knn synchronises
 *    (it needs the edge count).  Arguments are validated on the host before
 *    any device work, so invalid input never reaches a kernel.
 *  - Node and edge indices are int32: n < 2^31 and E < 2^31 per graph/batch.
 *  - Results are deterministic: no floating-point atomics are used, and the
 *    same inputs on the same device give bitwise identical outputs.
 */
#ifndef XMGN_H
#define XMGN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t xmgn_status;
#define XMGN_OK 0
#define XMGN_ERR_INVALID (-1)     /* bad argument or inconsistent sizes */
#define XMGN_ERR_OOM (-2)         /* device or host allocation failed */
#define XMGN_ERR_HIP (-3)         /* a HIP runtime call failed */
#define XMGN_ERR_CAPACITY (-4)    /* a caller buffer is too small */
#define XMGN_ERR_UNSUPPORTED (-5) /* hidden width / device not supported */
#define XMGN_ERR_STATE (-6)       /* call order violated (e.g. backward first) */

typedef void* xmgn_stream; /* hipStream_t */

typedef struct xmgn_ctx xmgn_ctx;         /* device context: workspace, tape */
typedef struct xmgn_graph xmgn_graph;     /* receiver-sorted CSR graph */
typedef struct xmgn_partset xmgn_partset; /* partitions with halos */

/* Message of the last failing call on this thread (never NULL). */
const char* xmgn_last_error(void);
/* Library version string. */
const char* xmgn_version(void);

/*
 * Model description.  Architecture (MeshGraphNet, Sec. II; X-MeshGraphNet
 * Sec. III.D):
 *   node encoder  node_in -> H -> H -> H, then LayerNorm
 *   edge encoder  edge_in -> H -> H -> H, then LayerNorm; the edge input is
 *                 [x_s - x_r, |x_s - x_r|] (Sec. II.E) normalised by a
 *                 caller-given affine
 *   n_layers processor layers (Eq. 1-4): per edge k = (s -> r)
 *       v_k = LN(W2e act(W1e [h_r; h_s; e_k] + b1e) + b2e),  e'_k = e_k + v_k
 *       m_r = sum of v_k over the in-edges of r (aggregate 0) or of e'_k
 *             (aggregate 1), added in ascending sender order
 *       h'_r = h_r + LN(W2n act(W1n [h_r; m_r] + b1n) + b2n)
 *   decoder H -> H -> H -> out_dim, no LayerNorm.
 *   LN(u) = gamma (u - mean) / sqrt(var + ln_eps) + beta, biased variance.
 */
typedef struct {
  int32_t hidden;     /* H: 128, 256, or 512 (BF16 form only) */
  int32_t n_layers;   /* processor layers L >= 1 */
  int32_t node_in;    /* node input width: 1..8, or a multiple of 4 up to 32
                         (6 = position + normal; 24 adds their Fourier features) */
  int32_t edge_in;    /* must be 4 */
  int32_t out_dim;    /* decoder outputs, 1..16 */
  int32_t activation; /* 0 = ReLU, 1 = SiLU */
  int32_t precision;  /* 0 = plain FP32 (FP32 storage, FP32 MFMA),
                         1 = BF16 storage and MFMA operands, FP32 accumulate,
                             FP32 LayerNorm statistics, segment sums and
                             gradient accumulation */
  int32_t aggregate;  /* 0 = sum of messages v, 1 = sum of updated edges e' */
  float ln_eps;       /* LayerNorm epsilon, e.g. 1e-5 */
} xmgn_model_desc;

/*
 * Parameter blob: FP32, flat, in this order, every W stored [out][in]:
 *   block 0 node encoder: W1[H][node_in] b1[H] W2[H][H] b2[H] W3[H][H] b3[H] gamma[H] beta[H]
 *   block 1 edge encoder: W1[H][edge_in] b1 W2 b2 W3 b3 gamma beta (as above)
 *   per layer l = 0..L-1:
 *     block 2 edge MLP:   W1[H][3H] b1[H] W2[H][H] b2[H] gamma[H] beta[H]
 *     block 3 node MLP:   W1[H][2H] b1[H] W2[H][H] b2[H] gamma[H] beta[H]
 *   block 4 decoder:      W1[H][H] b1[H] W2[H][H] b2[H] W3[out][H] b3[out]
 * xmgn_param_count gives the total; xmgn_param_offset the start of tensor
 * `tensor` (0-based, in the order above) of `block` (layer ignored for
 * blocks 0, 1, 4).
 */
xmgn_status xmgn_param_count(const xmgn_model_desc* desc, int64_t* count);
xmgn_status xmgn_param_offset(const xmgn_model_desc* desc, int32_t block, int32_t layer,
                              int32_t tensor, int64_t* offset);

/* Context on HIP device `device` (must be gfx950). */
xmgn_status xmgn_ctx_create(int32_t device, xmgn_ctx** out);
void xmgn_ctx_destroy(xmgn_ctx* ctx);

/* Tile configuration of the processor kernels: rows per tile of the edge
 * kernels (32, 64 or 128) and node kernels (32 or 64), the persistent grid
 * size in workgroups (a multiple of 8) and the waves per workgroup of the
 * edge kernels (4 or 8); 0 selects the library default for any of them (64,
 * 64, 1024, 4; at H = 512 8 edge waves and, in the BF16 gathered forward,
 * the wide kernel's 64-row tiles).  LDS fixes the rows at H = 128
 * (at most 64-row edge tiles), at H = 256 (32-row node tiles; 32-row edge
 * tiles unless, in the BF16 form, 64 are asked for, or 128 for the gathered
 * edge forward's wide kernel, 8 waves, whose edge adjoint then runs 64-row
 * tiles unless set otherwise) and at H = 512 (16-row node tiles; 32-row edge
 * tiles unless 64 are asked for the BF16 gathered forward's wide kernel,
 * whose adjoint stays on 32) whatever is asked.  Changing it invalidates
 * cached batch plans. */
xmgn_status xmgn_ctx_set_tiles(xmgn_ctx* ctx, int32_t edge_rows, int32_t node_rows,
                               int32_t grid, int32_t edge_waves);

/* Tiles of the edge adjoint, which tiles the same edges on its own (whole
 * receiver segments per tile).  edge_rows: 32 or 64 in the BF16 form at
 * H = 128 and 256 (at H = 128, 32-row tiles with the z tape run a variant
 * that keeps half the weight-gradient accumulators and two workgroups per
 * compute unit), else the forward's; 0 = the forward's.  edge_waves: 4 or 8
 * waves per workgroup, any form; 0 = the forward's.  Invalidates the last
 * forward. */
xmgn_status xmgn_ctx_set_bwd_tiles(xmgn_ctx* ctx, int32_t edge_rows, int32_t edge_waves);
xmgn_status xmgn_ctx_get_bwd_tiles(const xmgn_ctx* ctx, int32_t* edge_rows, int32_t* edge_waves);

/*
 * 1. Multi-scale kNN graph (Sec. III.B, III.C).
 * pos: dev float32 [n][3].  Level l is the prefix [0, level_end[l]) of the
 * points (level_end: host int32 [n_levels], strictly increasing, last == n).
 * Every point of level l receives an edge from each of its k_intra nearest
 * other points of level l, and (l >= 1) from each of its k_cross nearest
 * points of level l-1.  Distances are squared Euclidean in FP64 from the
 * FP32 coordinates, summed x, y, z in that order without fused
 * multiply-add; equal distances rank the lower index first; the point itself
 * is excluded by index.  Repeated (receiver, sender) pairs are kept once and
 * each receiver's senders are sorted ascending.  Requires k_intra <
 * level_end[0], k_cross < level_end[0], k_intra <= 16, k_cross <= 16.
 * Synchronises `stream` once.  The graph keeps a device and a host copy.
 */
xmgn_status xmgn_build_knn(xmgn_ctx* ctx, const float* pos, int32_t n, const int32_t* level_end,
                           int32_t n_levels, int32_t k_intra, int32_t k_cross, xmgn_graph** out,
                           xmgn_stream stream);
/* Graph from a host CSR (row_ptr int32 [n+1], col int32 [E] senders,
 * each segment strictly ascending).  Host-only; no device memory. */
xmgn_status xmgn_graph_from_csr(int32_t n, const int32_t* row_ptr, const int32_t* col,
                                xmgn_graph** out);
xmgn_status xmgn_graph_info(const xmgn_graph* g, int32_t* n_nodes, int64_t* n_edges);
/* Copy the CSR to host arrays row_ptr [n+1] and col [E]. */
xmgn_status xmgn_graph_export(const xmgn_graph* g, int32_t* row_ptr, int32_t* col);
void xmgn_graph_destroy(xmgn_graph* g);

/*
 * 2. Partitions with an L-hop halo (Sec. III.A), host-side.
 * pos: host float32 [n][3]; part_sizes: host int32 [n_parts], positive, sum n.
 * Recursive coordinate bisection: parts [a, b) split at m = a + (b-a)/2
 * along the axis of largest bounding-box extent (x, y, z on ties), nodes
 * ordered by (coordinate, id), the first sum(part_sizes[a:m]) go left.
 * The halo of a part is every node within halo_hops in-edge hops of it
 * (breadth-first over senders).  Local node order: inner nodes by id, then
 * halo nodes by (hop, id).  Local edges: all in-edges of local nodes with hop
 * < halo_hops, each segment in ascending global sender id.  With halo_hops
 * >= n_layers the inner outputs equal the full-graph outputs.
 */
xmgn_status xmgn_partition_halo(const xmgn_graph* g, const float* pos, int32_t n_parts,
                                const int32_t* part_sizes, int32_t halo_hops,
                                xmgn_partset** out);
/* Partitions given by an explicit inner-node list per part (host int32
 * arrays concatenated in `inner`, counts in `n_inner`), each extended by a
 * halo_hops halo.  Parts may overlap (e.g. in-cones of sampled nodes). */
xmgn_status xmgn_partition_explicit(const xmgn_graph* g, int32_t n_parts, const int32_t* n_inner,
                                    const int32_t* inner, int32_t halo_hops, xmgn_partset** out);
xmgn_status xmgn_partset_count(const xmgn_partset* ps, int32_t* n_parts, int32_t* n_global);
xmgn_status xmgn_partset_info(const xmgn_partset* ps, int32_t part, int32_t* n_inner,
                              int32_t* n_halo, int64_t* n_edges);
/* Host outputs of one part: global_ids [n_inner + n_halo] (local order),
 * hop [same], row_ptr [n_local + 1], col [n_edges] (local sender index).
 * Any output pointer may be NULL. */
xmgn_status xmgn_partset_export(const xmgn_partset* ps, int32_t part, int32_t* global_ids,
                                int32_t* hop, int32_t* row_ptr, int32_t* col);
void xmgn_partset_destroy(xmgn_partset* ps);

/*
 * 3. Forward over a batch of partitions (a whole graph is one partition with
 * halo 0).  The batch is the disjoint union of parts part_ids (host int32
 * [n_batch], distinct); its plan is built on the first call and cached.
 * params:    dev FP32 blob (layout above)
 * node_in:   dev FP32 [N_global][node_in]
 * pos:       dev FP32 [N_global][3]
 * edge_norm: host FP32 [2][edge_in]: mean then std of the edge input
 * out:       dev FP32 [N_global][out_dim]; only the rows of the batch's inner
 *            nodes are written (halo predictions are dropped, Sec. III.D)
 * keep_tape: 1 keeps per-layer checkpoints (h^l, e^l, m^l) for backward.
 * params and node_in must stay valid and unchanged until the matching
 * xmgn_backward has been enqueued: the backward re-reads them (the node
 * encoder is recomputed from its input; the edge encoder from the edge
 * features this call derives from pos and keeps in the context).
 */
xmgn_status xmgn_forward(xmgn_ctx* ctx, const xmgn_model_desc* desc, const float* params,
                         const xmgn_partset* ps, const int32_t* part_ids, int32_t n_batch,
                         const float* node_in, const float* pos, const float* edge_norm,
                         float* out, int32_t keep_tape, xmgn_stream stream);

/*
 * Masked MSE of the last forward (Sec. II.E; halo rows excluded, Sec. III.D):
 * loss = sum over the batch's inner nodes i and channels c of
 *        (out[i][c] - target[i][c])^2 / (n_total * out_dim),
 * d_out[i][c] = 2 (out - target) / (n_total * out_dim) on the same rows
 * (other rows untouched).  out, target, d_out: dev FP32 [N_global][out_dim];
 * loss: dev FP32 [1], overwritten.  n_total: the normaliser (the full
 * graph's node count, so partition losses add up to the full loss).
 */
xmgn_status xmgn_mse_grad(xmgn_ctx* ctx, const float* out, const float* target, int64_t n_total,
                          float* d_out, float* loss, xmgn_stream stream);

/*
 * 4. Backward of the last forward on ctx (which must have kept its tape):
 * the gradient of sum(d_out * out) with respect to every parameter, by the
 * hand-written adjoint of the encoders, the processor layers (Eq. 1-4) and
 * the decoder.
 * d_out: dev FP32 [N_global][out_dim]; only the rows of the batch's inner
 *        nodes are read (halo predictions are dropped, Sec. III.D, so they
 *        carry no gradient).
 * d_params: dev FP32, same layout as params; written, not added.
 * Gradient aggregation (Sec. III.A): each part's halo reproduces the
 * computational graph of its inner nodes, so the gradients of the parts of a
 * partition set (one backward per batch, summed with xmgn_grad_accumulate in
 * a fixed order) add up to the full graph's, as if the whole graph had been
 * processed; a batch of several parts returns that sum itself.
 * Activation checkpointing (Sec. V.D, V.F): the forward keeps only each
 * layer's input latents (h^l, e^l) and sums m^l; every layer's MLPs are
 * recomputed from them here, except that the BF16 forms may keep the edge
 * MLP's hidden activations (and, under SiLU, their pre-activations) when
 * the tape policy allows (xmgn_ctx_set_tape).
 * Errors: XMGN_ERR_STATE when ctx holds no tape, or desc or params differ
 * from the forward's; nothing is enqueued then.
 */
xmgn_status xmgn_backward(xmgn_ctx* ctx, const xmgn_model_desc* desc, const float* params,
                          const float* d_out, float* d_params, xmgn_stream stream);

/*
 * Tile autotuner (batching).  Times forward + backward of the batch over
 * candidate configurations -- edge-tile rows {32, 64} x edge waves {4, 8} x
 * persistent grid {4, 8} workgroups per compute unit, then node-tile rows
 * {32, 64} for the best of those (64-row edge tiles at H = 128 and, BF16,
 * H = 256; 64-row node tiles at H = 128), then the edge adjoint's own
 * waves {4, 8} and (BF16, H = 128 and 256) its own tile rows {32, 64}
 * against each edge-tile height and wave count of the forward -- and keeps
 * the fastest in ctx (as xmgn_ctx_set_tiles and xmgn_ctx_set_bwd_tiles
 * would).
 * Arguments as for xmgn_forward / xmgn_backward; out and d_params are
 * overwritten, d_out is only read.  cache_path (host string or NULL): a text
 * file of configuration lines; a hit skips the timing,
 * a miss appends a line ("key edge_rows node_rows grid edge_waves
 * adjoint_edge_rows adjoint_edge_waves ms").  The key holds the device name, the model
 * description, the tape policy and the batch's node and edge counts.  The chosen
 * configuration and its step time are returned (any output pointer may be
 * NULL).  Synchronises the stream.
 */
xmgn_status xmgn_autotune(xmgn_ctx* ctx, const xmgn_model_desc* desc, const float* params,
                          const xmgn_partset* ps, const int32_t* part_ids, int32_t n_batch,
                          const float* node_in, const float* pos, const float* edge_norm,
                          float* out, const float* d_out, float* d_params, const char* cache_path,
                          int32_t* edge_rows, int32_t* node_rows, int32_t* grid, int32_t* edge_waves,
                          float* step_ms, xmgn_stream stream);

/* 5. acc[i] += g[i] for i < n (dev FP32), elementwise, deterministic
 * (gradient aggregation over partitions, Sec. III.A). */
xmgn_status xmgn_grad_accumulate(float* acc, const float* g, int64_t n, xmgn_stream stream);

/*
 * Optimizer step of the paper's training (Sec. V.D: Adam, gradients clipped
 * at a global L2 norm of 32, learning rate annealed on a cosine).
 * params, m, v: dev FP32 [n], updated in place (m, v start at zero);
 * grad: dev FP32 [n], read only.  With clip_norm > 0 the gradient is first
 * scaled by min(1, clip_norm / (||grad||_2 + 1e-6)), the norm taken over
 * all n entries and summed in FP64 in a fixed order; then, with t = step
 * (1-based), m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2 and
 * params -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * grad_norm: dev FP32 [1] receiving ||grad||_2 before clipping, or NULL.
 * The update runs in FP32; the host scalars 1 - b1, 1 - b2, 1 - b1^t and
 * 1 - b2^t are formed in FP64 and rounded once.  Deterministic,
 * asynchronous on `stream`; uses a small scratch buffer of ctx, so steps on
 * one ctx must be ordered on one stream.  Errors: XMGN_ERR_INVALID for
 * step < 1, betas outside [0, 1), a non-finite or negative lr, eps <= 0.
 */
xmgn_status xmgn_adam_step(xmgn_ctx* ctx, float* params, const float* grad, float* m, float* v,
                           int64_t n, int64_t step, double lr, double beta1, double beta2, double eps,
                           double clip_norm, float* grad_norm, xmgn_stream stream);
/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training or serving loops, harnesses that forbid
 * hipMalloc): xmgn_adam_step without a context, allocating nothing.  Same
 * arguments, checks and kernels, and bitwise the same results; the clipping
 * norm's per-workgroup partials go to a fixed array of the library instead
 * of a context buffer: 256 FP64 values (2 KiB) on each GPU the library runs
 * on, held until the process ends.  The partial count does not grow with n,
 * so every n >= 0 fits.  device: the HIP device the arrays live on (made
 * current, like a context's calls do); its array's address is looked up on
 * the first call on that device.  Every call writes all 256 partials before
 * reading them, so nothing carries over from an earlier call; calls that
 * overlap on one GPU (other streams, other threads) race on the array:
 * order them on one stream.  Errors: as xmgn_adam_step, plus
 * XMGN_ERR_INVALID for a device index out of range.
 */
xmgn_status xmgn_adam_step_noalloc(int32_t device, float* params, const float* grad, float* m, float* v,
                                   int64_t n, int64_t step, double lr, double beta1, double beta2, double eps,
                                   double clip_norm, float* grad_norm, xmgn_stream stream);
/* Cosine-annealed learning rate (Sec. V.D) at step t of T (host, no device
 * work): lr_min + (lr_max - lr_min) (1 + cos(pi t / T)) / 2 with t clamped
 * to [0, T]; lr_min when T <= 0. */
double xmgn_cosine_lr(int64_t t, int64_t T, double lr_max, double lr_min);

/*
 * Per-kernel timing (tracing).  While enabled, every kernel the context
 * launches is bracketed by a pair of HIP events on its stream; the totals per
 * kernel class since the last xmgn_ctx_set_timing call are read with
 * xmgn_ctx_timing_read (which synchronises those events).  Do not enable it
 * while the stream is being captured into a graph.
 */
xmgn_status xmgn_ctx_set_timing(xmgn_ctx* ctx, int32_t enable);
xmgn_status xmgn_ctx_timing_count(const xmgn_ctx* ctx, int32_t* n_classes);
/* Class i: name (NUL-terminated, truncated to name_len), summed duration in
 * milliseconds and number of launches. */
xmgn_status xmgn_ctx_timing_read(xmgn_ctx* ctx, int32_t i, char* name, int32_t name_len, double* total_ms,
                                 int64_t* launches);

/*
 * Serial number of the tape the next xmgn_backward on ctx would consume: a
 * positive count of the forwards enqueued on ctx so far, taken at the last
 * one if it kept its tape, else 0 (no tape: no forward yet, the last forward
 * had keep_tape = 0 or failed, or the tiles or the offload mode changed
 * since).  A caller that holds several forwards open on one context (e.g.
 * an autograd graph over two partitions) records it after each forward and
 * compares it before the matching backward: a different value means a later
 * forward replaced the tape.  Host-only, never fails for a valid ctx.
 */
xmgn_status xmgn_ctx_tape_serial(const xmgn_ctx* ctx, int64_t* serial);

/* Device bytes currently held by the context (tape and workspace). */
xmgn_status xmgn_ctx_memory(const xmgn_ctx* ctx, int64_t* bytes);

/*
 * Activation checkpoints offloaded to host memory (Sec. V.F.1).  While
 * enabled, a forward with keep_tape = 1 keeps on the device only two
 * rotating slots of the per-layer checkpoints (h^l, e^l, m^l) and copies
 * each layer's checkpoint into page-locked host memory owned by the context,
 * on a copy stream of its own, overlapped with the next layer (a layer waits
 * only for the copies of the layer two before it).  The backward copies
 * layer l-1's checkpoint back while layer l runs.  The hidden activations of
 * the edge MLP (and their pre-activations) are never offloaded: the edge
 * adjoint recomputes them.  The
 * checkpoints of the last two layers stay in their device slots and are not
 * copied.  Results equal those of the device-resident tape up to the
 * recomputed hidden activations (bitwise in the FP32 form, whose
 * device-resident tape recomputes them too).  Enabling or disabling synchronises the device,
 * frees the current tape (it is re-allocated at its new size by the next
 * forward) and invalidates the last forward.  The forward completes (on its
 * stream) only when its host copies have landed; each call's copies stay
 * ordered with its own stream, so the usual stream rules apply.  Pinned
 * bytes: ((L+1) n + L E) H s + 4 L n H for a batch of n nodes and E edges,
 * s = 2 (BF16) or 4 (FP32).
 */
xmgn_status xmgn_ctx_set_offload(xmgn_ctx* ctx, int32_t enable);
/*
 * Tape policy of the training forward (activation checkpointing, Sec. V.D,
 * V.F).  keep_hidden = 0: the tape holds each layer's checkpoints only
 * (h^l, e^l, m^l) and the backward recomputes both products of every edge
 * MLP from them.  keep_hidden = 1 (the default): the tape also keeps every
 * edge's hidden activation z = act(a) of every layer, stored like the
 * latents (BF16 or FP32; under SiLU also a), L E H s bytes each, and the
 * edge adjoint reads it instead of recomputing the first product; the
 * offloaded tape always recomputes.  Both policies give the same forward
 * outputs bitwise; their gradients agree to the rounding of the stored z
 * (the recompute may sum the first product in another order, and SiLU's
 * derivative is taken at the stored pre-activation).  Changing it
 * synchronises the device, frees the hidden-activation tape and
 * invalidates the last forward.
 */
xmgn_status xmgn_ctx_set_tape(xmgn_ctx* ctx, int32_t keep_hidden);
xmgn_status xmgn_ctx_get_tape(const xmgn_ctx* ctx, int32_t* keep_hidden);
/*
 * Form of the edge forward (Eq. 1).  split = 0 (the default): every edge
 * gathers [h_r ; h_s ; e] into LDS and applies the 3H -> H first layer.
 * split = 1: the first layer is re-associated over its input blocks,
 * W1 x + b1 = W1_e e + (W1_r h_r + b1) + W1_s h_s; a per-node kernel first
 * computes W1_r h + b1 and W1_s h for every node of the batch (FP32,
 * 8 n H bytes of context memory), and each edge then adds the rows of its
 * receiver and sender to W1_e e.  The value is the same up to the rounding
 * order of the sum; the product's flops per edge fall from 6 H^2 to 2 H^2.
 * The split form runs in forwards without a tape and in forwards whose tape
 * keeps z (keep_hidden = 1, resident); elsewhere the gathered form runs, so
 * that an adjoint that recomputes the first product sees the forward's own
 * rounding.  Invalidates the last forward.
 */
xmgn_status xmgn_ctx_set_edge_split(xmgn_ctx* ctx, int32_t split);
xmgn_status xmgn_ctx_get_edge_split(const xmgn_ctx* ctx, int32_t* split);
/* Page-locked host bytes currently held by the context (the offloaded tape). */
xmgn_status xmgn_ctx_host_memory(const xmgn_ctx* ctx, int64_t* bytes);

#ifdef __cplusplus
}
#endif

#endif /* XMGN_H */
