/*
 * spx.h -- C ABI of libspx.so: the multiresolution simplex hash encoding of
 * Wen & Yang, "Efficient Encoding of Graphics Primitives with Simplex-based
 * Structures" (arXiv 2311.15439), on AMD Instinct MI355X (gfx950).
 *
 * Conventions shared by every entry point
 *   - Pointers documented "device" address GPU memory owned by the caller
 *     (for example torch tensors); pointers documented "host" address CPU
 *     memory read or written during the call only.  The library never
 *     allocates, frees or keeps a pointer after returning; its only device
 *     memory of its own is the static scratch of spx_mlp_bwd_noalloc.
 *   - Calls that take a hipStream_t enqueue their kernels on that stream and
 *     return without waiting.  Argument checks happen on the host before
 *     anything is enqueued; a call that returns an error has enqueued
 *     nothing (SPX_EHIP excepted: the launch itself failed).
 *   - Every call returns spx_status; no C++ exception crosses the ABI.
 *     spx_last_error() gives a human-readable detail of the last failure on
 *     the calling thread.
 *   - N = 0 (no points) is a valid no-op that returns SPX_OK.
 *   - Calls are stateless and thread-safe; results are deterministic except
 *     where an entry point accumulates with atomics (noted below).
 *   - Dtype codes: SPX_F32 = IEEE binary32, SPX_F16 = IEEE binary16.
 */
#ifndef SPX_H_
#define SPX_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPX_ABI_VERSION 2
#define SPX_MAX_DIMS 6
#define SPX_MAX_LEVELS 32
#define SPX_MAX_LOG2_T 26

typedef enum {
    SPX_OK = 0,
    SPX_EINVAL = 1,       /* bad shape, size, dtype, flag or null pointer */
    SPX_EALIGN = 2,       /* a device pointer lacks the documented alignment */
    SPX_EUNSUPPORTED = 3, /* well-formed request outside what is built */
    SPX_EHIP = 4          /* the HIP runtime reported an error at launch */
} spx_status;

enum { SPX_F32 = 0, SPX_F16 = 1 };
enum { SPX_SIMPLEX = 0, SPX_GRID = 1 };
enum { SPX_LAYOUT_HASHED = 0, SPX_LAYOUT_SIZED = 1 };

/*
 * Encoding descriptor (host memory, read during the call only).
 *   n_dims       n, 1..6: dimension of the input points.
 *   n_levels     L, 1..32: number of resolution levels.
 *   log2_T       each level's table has T = 2^log2_T entries, 1..26.
 *   n_feat       F, 1, 2, 4 or 8: features per table entry.
 *   table_dtype  SPX_F32 or SPX_F16.
 *   cell         SPX_SIMPLEX (the paper's method: n+1 vertices per level)
 *                or SPX_GRID (the 2^n-corner multilinear baseline).
 *   equal_memory 0 or 1: scale every level's resolution by
 *                (n+1)^((n-1)/(2n)), the factor the paper uses to compare
 *                simplex and grid at the same table size (Sec. 5.2).
 *                Ignored for SPX_GRID.
 *   res[l]       N_l >= 1, the resolution of level l (l < n_levels).
 *   layout       how each level's vertices map to table rows (Sec. 5.2,
 *                Hash Table Selection):
 *                SPX_LAYOUT_HASHED: every level has T rows and every vertex
 *                  is hashed (the paper's configurations);
 *                SPX_LAYOUT_SIZED: the box of vertices the closed unit cube
 *                  reaches at level l has ext_l^n vertices (ext_l from
 *                  spx_table_layout).  If that is at most T, the level is
 *                  stored densely: ext_l^n rows, vertex v at row
 *                  sum_i v_i ext_l^i (no collisions; the coordinates of
 *                  points outside the cube are clamped to the box).
 *                  Otherwise it is hashed into the
 *                  smallest power of two of rows that holds the share of
 *                  the box a simplex level uses, (n+1)^(-(n-1)/2) (all of it
 *                  for the grid), at most T.
 * Tables are laid out level after level, feature innermost: level l's rows
 * start at row offset_l = rows_0 + ... + rows_{l-1} (spx_table_layout); for
 * SPX_LAYOUT_HASHED that is [L][T][F].  The encoded features are [N][L*F]
 * (levels concatenated in order, Sec. 5 step (d)).
 */
typedef struct {
    int32_t n_dims;
    int32_t n_levels;
    int32_t log2_T;
    int32_t n_feat;
    int32_t table_dtype;
    int32_t cell;
    int32_t equal_memory;
    int32_t res[SPX_MAX_LEVELS];
    int32_t layout;
} spx_encoding;

/* ABI version compiled into the library (SPX_ABI_VERSION). */
int32_t spx_abi_version(void);

/* Static string naming a status code. */
const char* spx_status_str(spx_status s);

/* Detail of the most recent failure on the calling thread ("" if none). */
const char* spx_last_error(void);

/*
 * Kernel tracing (profiling aid).  While a trace is set on a thread, every
 * kernel the library launches from that thread is bracketed by
 * events[2i] / events[2i+1], recorded on its launch stream, and described
 * by names[i] (a static string) and bytes[i] (the bytes the kernel must move
 * by its own definition: inputs read plus outputs written).  Kernels beyond
 * capacity are not recorded.  With `only` set, only kernels of that name are
 * recorded (the others run without events around them).  The caller creates
 * the 2 * capacity events and reads the elapsed times after synchronising.
 * Pass NULL to stop.
 */
typedef struct {
    hipEvent_t* events;   /* [2 * capacity] */
    const char** names;   /* [capacity] */
    double* bytes;        /* [capacity] */
    int32_t capacity;
    int32_t count;        /* kernels recorded so far (written by the library) */
    const char* only;     /* NULL: every kernel; else the one kernel name to record */
} spx_trace;

spx_status spx_trace_set(spx_trace* trace);

/*
 * Host helper: geometric level schedule N_l = floor(n_min * growth^l + 1e-6)
 * for l < L (the paper scales the unit cube per level, Sec. 5.1, without
 * fixing the schedule).  res_out: host [L].  Errors: SPX_EINVAL if
 * L is outside 1..32, n_min < 1, growth < 1 or res_out is NULL.
 */
spx_status spx_level_resolutions(double n_min, double growth, int32_t L, int32_t* res_out);

/*
 * Host helper: the binary32 multiplier sigma_l that the kernels apply to a
 * point at level l.  Simplex: sigma_l = N_l * c / sqrt(n+1), evaluated in
 * binary64 and rounded once, where sqrt(n+1) is the adjustment scale S_n
 * that maps the skewed unit cube [0, S_n]^n back to [0,1]^n (Sec. 5.1) and c
 * is the equal-memory factor or 1.  Grid: sigma_l = N_l.
 * sigma_out: host [n_levels].
 */
spx_status spx_level_scales(const spx_encoding* enc, float* sigma_out);

/*
 * Host helper: the table layout of an encoding (Sec. 5.2).  Per level
 * (host arrays of n_levels entries, each may be NULL): level_rows, the rows
 * of its table; box_extent, the extent per axis of the vertex box the
 * closed unit cube reaches (the far corner (1,...,1) skewed and scaled in
 * binary32, floored, plus 2); dense, 1 if the level is stored densely.
 * *total_rows (may be NULL): rows of all levels; the tables hold
 * total_rows * n_feat values.
 */
spx_status spx_table_layout(const spx_encoding* enc, int64_t* level_rows, int32_t* box_extent, int32_t* dense,
                            int64_t* total_rows);

/*
 * Host helper: the six hash multipliers P_0..P_5.  A vertex v of level l is
 * stored at slot (XOR_i uint32(v_i) * P_i mod 2^32) & (T - 1) of that
 * level's table (Sec. 5 steps (a)-(b); the paper does not print its hash).
 * primes_out: host [6].
 */
spx_status spx_hash_primes(uint32_t* primes_out);

/*
 * Forward encoding (Sec. 5 steps (a)-(d); Secs. 4.1-4.3 for the simplex).
 * Per point: skew (Eq. 2), then per level scale by sigma_l, split into
 * lattice cell and fractional part, order the fractions largest first (ties
 * to the lower axis) to pick the simplex, walk its n+1 vertices, weight
 * them barycentrically, hash them, and sum the weighted table rows.
 *   N        number of points, >= 0.
 *   pts      device [N][n] binary32, 4-byte aligned.  Any finite value is
 *            legal (the hash is total); positions are exact for
 *            |sigma_l * skewed coordinate| < 2^24.
 *   tables   device, the table layout's rows (spx_table_layout) of F
 *            values of enc->table_dtype, aligned to one row (F * element
 *            size, at most 16 bytes).
 *   out      device [N][L*F] of out_dtype (SPX_F32 or SPX_F16), aligned to
 *            F * element size (at most 16 bytes).  Overwritten.
 * Deterministic: the same inputs give bit-identical outputs.  From three
 * dimensions and 2^18 points, when the levels' reachable rows exceed an
 * XCD's 4 MiB L2 together but fit one by one, the launch is level-major:
 * groups of consecutive levels up to 4 MiB, one group after the other over
 * all points (the same outputs, faster).
 */
spx_status spx_encode_fwd(const spx_encoding* enc, int64_t N, const float* pts, const void* tables,
                          void* out, int32_t out_dtype, hipStream_t stream);

/*
 * Adjoint of spx_encode_fwd (Sec. 5 step (e)): for every point, level and
 * vertex, d_tables[l][h][j] += w * d_out[pt][l*F + j] with the forward's
 * weights and slots.  There is no gradient with respect to the points.
 *   d_out      device [N][L*F] of d_out_dtype (SPX_F32 or SPX_F16), aligned
 *              to F * element size (at most 16 bytes).
 *   d_tables   device binary32, laid out as the tables, 4-byte aligned.  ACCUMULATED: the
 *              caller zeroes it.  The summation order, and so the last bits,
 *              vary from run to run.
 *   workspace  NULL: every contribution is added with a binary32 atomic.
 *              Otherwise device memory of at least the size returned by
 *              spx_encode_bwd_workspace(), 256-byte aligned: contributions
 *              are first binned by slot range and summed in LDS, and each
 *              slot of d_tables is then updated by exactly one workgroup
 *              (no global atomics; much faster for large batches).  A
 *              bucket of slots that would hold more than one CU's share of
 *              the contributions (a small table with many contributions) is
 *              summed by several workgroups into partial sums that a second
 *              pass adds in a fixed order.
 *              workspace_bytes is its size.  Its contents on entry are
 *              ignored and on return undefined.
 */
spx_status spx_encode_bwd(const spx_encoding* enc, int64_t N, const float* pts, const void* d_out,
                          int32_t d_out_dtype, float* d_tables, void* workspace, size_t workspace_bytes,
                          hipStream_t stream);

/*
 * Workspace bytes the binned adjoint needs for N points (written to
 * *bytes): about N * L * V records of 8 to 64 bytes, per-bucket counters,
 * the privatised coarse levels' per-workgroup sums and the split buckets'
 * partial sums.  SPX_EUNSUPPORTED if the configuration cannot be binned (use the
 * atomic path, workspace NULL).
 */
spx_status spx_encode_bwd_workspace(const spx_encoding* enc, int64_t N, size_t* bytes);

/*
 * Adjoint and optimizer in one pass: the table gradient of spx_encode_bwd
 * (as if accumulated into a zeroed table) is summed per slot in LDS and the
 * Adam step of spx_adam_step is applied to every entry of the tables at
 * once, so no gradient table is written or read.  Every entry is updated
 * (entries with zero gradient still decay m and v), exactly as
 * spx_encode_bwd into zeros followed by spx_adam_step over all total_rows*F
 * entries.
 *   param, m, v  device binary32 laid out as the tables, 16-byte aligned:
 *                master tables and Adam moments, updated in place.
 *   param_f16    device binary16 laid out as the tables, 8-byte aligned, or
 *                NULL: receives
 *                the binary16 image of the updated tables (the forward's
 *                input).
 *   lr, beta1, beta2, eps, step   as spx_adam_step.
 *   workspace    as spx_encode_bwd (required here), 256-byte aligned.
 */
spx_status spx_encode_bwd_adam(const spx_encoding* enc, int64_t N, const float* pts, const void* d_out,
                               int32_t d_out_dtype, float* param, float* m, float* v, uint16_t* param_f16,
                               float lr, float beta1, float beta2, float eps, int64_t step, void* workspace,
                               size_t workspace_bytes, hipStream_t stream);

/*
 * The part of the binned adjoint (Sec. 5 step (e)) that depends only on the
 * points: which slot range each contribution falls in, counted per
 * workgroup of the adjoint's scatter and turned into every record's place
 * in the workspace (for the first level group; a configuration with more
 * than one group counts the others in the adjoint call itself).  It exists
 * so that a caller can issue it on a second stream while the forward and
 * the network run (it needs no gradient), and then call
 * spx_encode_bwd_prepared or spx_encode_bwd_adam_prepared, which skip it.
 *   pts, N      the points the adjoint will be called with.
 *   workspace   as spx_encode_bwd (required), 256-byte aligned; the
 *               prepared adjoint must get the same workspace, encoding, N
 *               and unchanged points, and the caller orders the two calls
 *               (an event recorded after this call on its stream, waited on
 *               by the adjoint's stream), and keeps other adjoint calls
 *               that use this workspace from running in between.
 * N = 0 is a no-op.
 */
spx_status spx_encode_bwd_prepare(const spx_encoding* enc, int64_t N, const float* pts, void* workspace,
                                  size_t workspace_bytes, hipStream_t stream);

/*
 * spx_encode_bwd (binned: workspace required) after spx_encode_bwd_prepare
 * on the same encoding, N, points and workspace: the same result, without
 * the counting it did.
 */
spx_status spx_encode_bwd_prepared(const spx_encoding* enc, int64_t N, const float* pts, const void* d_out,
                                   int32_t d_out_dtype, float* d_tables, void* workspace, size_t workspace_bytes,
                                   hipStream_t stream);

/*
 * spx_encode_bwd_adam after spx_encode_bwd_prepare on the same encoding, N,
 * points and workspace: the same result, without the counting it did.
 */
spx_status spx_encode_bwd_adam_prepared(const spx_encoding* enc, int64_t N, const float* pts, const void* d_out,
                                        int32_t d_out_dtype, float* param, float* m, float* v, uint16_t* param_f16,
                                        float lr, float beta1, float beta2, float eps, int64_t step, void* workspace,
                                        size_t workspace_bytes, hipStream_t stream);

/*
 * Lookup introspection for parity tests: the slot and the binary32 weight
 * of every vertex, from the same code the forward and adjoint use.
 *   idx  device [N][L][V] uint32 slots (V = n+1, or 2^n for the grid whose
 *        corners are listed in binary order, bit i standing for axis i).
 *   w    device [N][L][V] binary32 weights.  Simplex vertices are listed in
 *        walk order: the cell corner first, then one step along the axis of
 *        each next-largest fraction.
 * Either output may be NULL.
 */
spx_status spx_encode_debug(const spx_encoding* enc, int64_t N, const float* pts, uint32_t* idx,
                            float* w, hipStream_t stream);

/*
 * Gradient of the encoding with respect to the input points, contracted
 * with the output gradient: d_pts[i] = sum over levels and features of
 * d_out * d out / d x_i.  Inside a simplex the weights are affine in the
 * fractional parts (Sec. 4.3): the derivative along the axis of the walk's
 * k-th step is the difference of the rows of vertices k+1 and k; it is
 * chained through p = sigma_l * skew(x) (Eq. 2).  The grid cell
 * differentiates its n-linear weights.  On a face, the one-sided derivative
 * of the simplex (or cell) the lookup picks is returned.
 *   tables  as spx_encode_fwd.
 *   d_out   device [N][L*F] binary32 or binary16 (d_out_dtype), row-aligned.
 *   d_pts   device [N][n] binary32, 4-byte aligned, overwritten.
 */
spx_status spx_encode_input_grad(const spx_encoding* enc, int64_t N, const float* pts, const void* tables,
                                 const void* d_out, int32_t d_out_dtype, float* d_pts, hipStream_t stream);

/*
 * Gather twin: a measurement reference for the forward, not part of the
 * method.  It streams the same points, finds the same cell at every level
 * and gathers the same number of table rows with the same per-level
 * locality (n+1 rows for the simplex, 2^n for the grid), but the simplex
 * walk takes the axes in index order (no sorting of the fractions) and the
 * rows are summed without weights.  Its throughput is the gather rate the
 * memory system sustains on the forward's access pattern; the forward's
 * rate divided by it is the forward's fraction of that gather roofline.
 *   tables  device [L][T][2] binary16 (n_feat must be 2, table_dtype
 *           SPX_F16, layout SPX_LAYOUT_HASHED), 4-byte aligned.
 *   out     device [N][L*2] binary16, 4-byte aligned: per level, the
 *           unweighted sum of the gathered rows.
 * Other feature counts or table types return SPX_EUNSUPPORTED.
 */
spx_status spx_encode_gather_twin(const spx_encoding* enc, int64_t N, const float* pts, const void* tables,
                                  void* out, hipStream_t stream);

/*
 * Random-gather probe: a measurement reference, not part of the method.
 * Each of n_threads threads gathers per_thread 4-byte words of `table` at
 * independent, uniformly random word offsets in [0, n_words) (a
 * counter-based hash of seed, thread and k; 16 loads in flight per
 * thread) and writes their 32-bit integer sum to out[thread].  The rate
 * at a buffer size is the memory system's random-access gather rate for
 * that footprint (cache level), the ceiling against which the encoding's
 * gathers, whose rows of one level are hashed uniformly over that level's
 * table (Sec. 5 steps (a)-(b)), are reported.
 *   table       device, 4-byte aligned, n_words words (n_words a power of
 *               two, 1..2^32).
 *   n_threads   0..2^30.
 *   per_thread  a multiple of 16 in 16..4096.
 *   out         device [n_threads] uint32, 4-byte aligned, overwritten.
 */
spx_status spx_gather_probe(const void* table, int64_t n_words, int64_t n_threads, int32_t per_thread,
                            uint32_t seed, uint32_t* out, hipStream_t stream);

/* Round-to-nearest-even binary32 -> binary16 copy of n elements (device,
 * src 4-byte and dst 2-byte aligned). */
spx_status spx_cast_f32_f16(int64_t n, const float* src, uint16_t* dst, hipStream_t stream);

/*
 * One Adam step (Kingma & Ba 2015, Algorithm 1; the paper trains by
 * gradient descent without naming the optimizer) on n binary32 parameters,
 * with bias correction for the 1-based iteration count `step`:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   param -= lr * (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).
 * All arrays are device binary32 [n], 4-byte aligned.  If param_f16 is not
 * NULL it receives the binary16 image of the updated parameters (the table
 * the forward gathers from).  If zero_grad is 1, grad is set to 0 after it
 * is read, ready for the next accumulation.
 */
spx_status spx_adam_step(int64_t n, float* param, float* grad, float* m, float* v, uint16_t* param_f16,
                         float lr, float beta1, float beta2, float eps, int64_t step, int32_t zero_grad,
                         hipStream_t stream);

/*
 * Gradient of the mean squared error loss of Sec. 6 (an L2 loss against the
 * target): d_y = scale * (y - target) elementwise over n values, with
 * scale = 2 / n for the mean.  y, target, d_y: device binary32 [n], 4-byte
 * aligned; d_y may alias y.
 */
spx_status spx_mse_grad(int64_t n, const float* y, const float* target, float* d_y, float scale,
                        hipStream_t stream);

/*
 * Volume rendering of ray samples (Sec. 6, Eq. 5): the rendering integral
 * evaluated over each ray's samples with the per-sample quadrature
 *   sigma_k = softplus(raw_k0), c_k = sigmoid(raw_k1..3),
 *   alpha_k = 1 - exp(-sigma_k delta_k),
 *   T_k = exp(-(sigma_0 delta_0 + ... + sigma_{k-1} delta_{k-1})),
 *   rgba = (sum_k T_k alpha_k c_k, sum_k T_k alpha_k)
 * (the last component is the ray's opacity; the activations are a reading,
 * the paper names none).  Binary32 arithmetic.
 *   n_rays     R >= 0 (0 is a no-op).
 *   n_samples  S, 1..1024 (SPX_EUNSUPPORTED otherwise), samples of one ray
 *              in order along the ray.
 *   raw        device [R*S][4] binary32, 16-byte aligned: the network's raw
 *              (density, r, g, b) per sample, ray-major.
 *   delta      device [R*S] binary32, 4-byte aligned: each sample's segment
 *              length along its ray.
 *   rgba       device [R][4] binary32, 16-byte aligned, overwritten.
 */
spx_status spx_composite_fwd(int64_t n_rays, int32_t n_samples, const float* raw, const float* delta, float* rgba,
                             hipStream_t stream);

/*
 * Adjoint of spx_composite_fwd: given d_rgba (device [R][4] binary32,
 * 16-byte aligned), writes d_raw (device [R*S][4] binary32, 16-byte
 * aligned, overwritten) = d rgba / d raw contracted with d_rgba.  The
 * forward quantities are recomputed from raw and delta (nothing is saved
 * between the calls).  Same argument rules as the forward.
 */
spx_status spx_composite_bwd(int64_t n_rays, int32_t n_samples, const float* raw, const float* delta,
                             const float* d_rgba, float* d_raw, hipStream_t stream);

/*
 * Tiny fully connected network of Sec. 5 step (e): d_in -> hidden -> hidden
 * -> d_out, ReLU after the two hidden layers, linear output.
 *   d_in    32 (the concatenated features, L*F; other widths return
 *           SPX_EUNSUPPORTED).
 *   hidden  64.
 *   d_out   1..16.
 * Weights are binary16, row-major, device, 16-byte aligned:
 * W1 [hidden][d_in], W2 [hidden][hidden], W3 [d_out][hidden].
 */
typedef struct {
    int32_t d_in;
    int32_t hidden;
    int32_t d_out;
} spx_mlp;

/*
 * Forward pass.  x: device [N][d_in] binary16, 16-byte aligned;
 * y: device [N][d_out] binary32, 4-byte aligned, overwritten.  Products run
 * on the matrix cores in binary16 with binary32 accumulation; hidden
 * activations are rounded to binary16.  Deterministic.
 */
spx_status spx_mlp_fwd(const spx_mlp* mlp, int64_t N, const uint16_t* x, const uint16_t* W1,
                       const uint16_t* W2, const uint16_t* W3, float* y, hipStream_t stream);

/*
 * Workspace needed by spx_mlp_bwd for N points (bytes, written to *bytes).
 */
spx_status spx_mlp_bwd_workspace(const spx_mlp* mlp, int64_t N, size_t* bytes);

/*
 * Backward pass (recomputes the forward).  d_y: device [N][d_out] binary32.
 * d_x: device [N][d_in] binary32, overwritten, or NULL to skip.
 * dW1/dW2/dW3: device binary32 with the weights' shapes, OVERWRITTEN with
 * the gradient summed over the N points.  Gradient operands are rounded to
 * bfloat16 for the matrix cores (binary32 accumulation); the ReLU mask is
 * taken on the stored binary16 activation.  workspace: device, at least
 * spx_mlp_bwd_workspace() bytes, 256-byte aligned.  The weight-gradient
 * sum is reduced in a fixed order: deterministic.
 */
spx_status spx_mlp_bwd(const spx_mlp* mlp, int64_t N, const uint16_t* x, const uint16_t* W1,
                       const uint16_t* W2, const uint16_t* W3, const float* d_y, float* d_x, float* dW1,
                       float* dW2, float* dW3, void* workspace, size_t workspace_bytes,
                       hipStream_t stream);

/*
 * spx_mlp_bwd without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The weight-gradient partials go
 * to a scratch array that the library holds in static device memory: 14 MiB
 * per GPU (the partials of the 512 workgroups the backward launches at
 * most), kept until the process ends.  Its device address is looked up
 * with hipGetSymbolAddress on the first call on each device; the call
 * itself allocates nothing.  Every N accepted by spx_mlp_bwd fits
 * (SPX_EUNSUPPORTED otherwise).  Every partial the reduction reads is
 * written by the same call, so nothing needs clearing; but all calls on one
 * GPU share the array, so calls that overlap in time on one GPU (on
 * different streams, or from different threads without ordering) race and
 * give wrong gradients: serialise them.  Results are bit-identical to
 * spx_mlp_bwd.  Other arguments and errors as spx_mlp_bwd.
 */
spx_status spx_mlp_bwd_noalloc(const spx_mlp* mlp, int64_t N, const uint16_t* x, const uint16_t* W1,
                               const uint16_t* W2, const uint16_t* W3, const float* d_y, float* d_x, float* dW1,
                               float* dW2, float* dW3, hipStream_t stream);

/*
 * Serving: several resident fields (encoding + network), queried together.
 *
 * spx_field is a device-ready descriptor of one field, filled on the host by
 * spx_field_init() (which also computes the level multipliers) and copied by
 * the caller into a device array.  Supported fields: n_dims 2 or 3, 16
 * levels of 2 binary16 features (32 network inputs), hidden width 64,
 * d_out 1..16, simplex or grid cells.
 */
typedef struct {
    float sigma[SPX_MAX_LEVELS]; /* binary32 level multipliers */
    float Fn;                    /* skew factor F_n (binary32) */
    uint32_t mask;               /* T - 1 */
    int32_t n_dims;
    int32_t n_levels;
    int32_t cell;
    int32_t d_out;
    const void* tables;          /* device [16][T][2] binary16, 4-byte aligned */
    const uint16_t* W1;          /* device [64][32] binary16, 16-byte aligned */
    const uint16_t* W2;          /* device [64][64] binary16 */
    const uint16_t* W3;          /* device [d_out][64] binary16 */
} spx_field;

/*
 * One segment of a batched query: count points of one field.
 *   pts         device [count][n_dims] binary32, 4-byte aligned
 *   out         device [count][d_out] binary32, overwritten
 *   first_tile  sum of ceil(count / 16) over all earlier segments of the
 *               batch (segments are processed in 16-point tiles)
 *   field       index into the fields array; a segment with an index
 *               outside [0, nfields) is skipped (its out is not written)
 */
typedef struct {
    const float* pts;
    float* out;
    int64_t count;
    int64_t first_tile;
    int32_t field;
    int32_t pad;
} spx_segment;

/*
 * Host helper: validate a field and fill *out (host memory).  enc must be a
 * 2- or 3-D encoding with 16 levels, 2 features and binary16 tables in the
 * hashed layout (SPX_EUNSUPPORTED otherwise).
 */
spx_status spx_field_init(const spx_encoding* enc, const void* tables, const uint16_t* W1, const uint16_t* W2,
                          const uint16_t* W3, int32_t d_out, spx_field* out);

/*
 * Encoding forward and network forward for every point of every segment, in
 * one launch (Sec. 5 steps (a)-(e) at inference).  fields: device
 * [nfields]; segs: device [nseg] with consistent first_tile values and
 * total_tiles = sum of ceil(count / 16).  Results are bit-identical to
 * spx_encode_fwd (binary16 features) followed by spx_mlp_fwd, whatever the
 * batch composition.  Inconsistent first_tile values cannot make the kernel
 * access memory outside a segment's pts/out ranges, but some points may then
 * not be computed.
 */
spx_status spx_field_query_batched(const spx_field* fields, int32_t nfields, const spx_segment* segs, int32_t nseg,
                                   int64_t total_tiles, hipStream_t stream);

/*
 * Encoding forward and network forward in one kernel, for training (Sec. 5
 * steps (a)-(e) forward): the same configurations as spx_field_init (2- or
 * 3-D, 16 levels of 2 binary16 features, a 32-64-64-d_out network, d_out
 * 1..16).  Per 16-point tile each lane encodes four levels of one point,
 * which are exactly its operand of the network's first matrix product, so
 * the features go from the gathers to the matrix cores in registers; they
 * are also stored (if feats is not NULL) for the network's backward.  When
 * feats is given and the level-major forward of spx_encode_fwd applies
 * (3-D, at least 2^18 points, each group of levels fits an XCD's L2 while
 * all levels together do not), the call runs spx_encode_fwd and
 * spx_mlp_fwd instead, which is faster there; the results are the same.
 *   feats  device [N][32] binary16, 16-byte aligned, or NULL: identical to
 *          spx_encode_fwd with a binary16 output.
 *   out    device [N][d_out] binary32, 4-byte aligned: identical to
 *          spx_mlp_fwd of those features.
 * Other arguments as spx_encode_fwd and spx_mlp_fwd; unsupported
 * configurations return SPX_EUNSUPPORTED.
 */
spx_status spx_encode_mlp_fwd(const spx_encoding* enc, const spx_mlp* mlp, int64_t N, const float* pts,
                              const void* tables, const uint16_t* W1, const uint16_t* W2, const uint16_t* W3,
                              uint16_t* feats, float* out, hipStream_t stream);

/*
 * Network backward and encoding adjoint with the tables' Adam step, fused
 * (Sec. 5 steps (d)-(e) backward): the result of spx_mlp_bwd (with d_x)
 * followed by spx_encode_bwd_adam of that d_x, without the input gradient
 * d_x ever being stored.  The adjoint's scatter computes each point's
 * input gradient itself on the matrix cores, from the stored features and
 * the network's output gradient, with the same products as spx_mlp_bwd (the
 * same bits), and emits its records from registers; only the units of the
 * privatised coarse levels (whose dense per-workgroup sums run beside the
 * scatter) are written to the workspace by the network backward.
 * Covered: the network's input is the encoding (d_in = n_levels * n_feat =
 * 32), n_feat = 2, n_dims 1..3, an adjoint that runs in one level group
 * (at most 16384 buckets and 2 GiB of records) with a staged scatter whose
 * LDS, with the network's weights, fits the CU; otherwise SPX_EUNSUPPORTED,
 * before anything is launched.
 *   x            device [N][32] binary16 features (the forward's), 16-byte aligned.
 *   W1, W2, W3   device binary16 weights as spx_mlp_fwd, 16-byte aligned.
 *   d_y          device [N][d_out] binary32 output gradient, 4-byte aligned.
 *   dW1..dW3     as spx_mlp_bwd: OVERWRITTEN with the weight gradients
 *                (deterministic, bit-identical to spx_mlp_bwd).
 *   param, m, v, param_f16, lr, beta1, beta2, eps, step
 *                as spx_encode_bwd_adam (every table entry takes its step).
 *   workspace    device, at least spx_encode_mlp_bwd_workspace() bytes,
 *                256-byte aligned; contents on entry ignored, on return
 *                undefined.
 * The tables' summation order varies from run to run, as in
 * spx_encode_bwd_adam.
 */
spx_status spx_encode_mlp_bwd_adam(const spx_encoding* enc, const spx_mlp* mlp, int64_t N, const float* pts,
                                   const uint16_t* x, const uint16_t* W1, const uint16_t* W2, const uint16_t* W3,
                                   const float* d_y, float* dW1, float* dW2, float* dW3, float* param, float* m,
                                   float* v, uint16_t* param_f16, float lr, float beta1, float beta2, float eps,
                                   int64_t step, void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Workspace bytes spx_encode_mlp_bwd_adam needs for N points (written to
 * *bytes): the binned adjoint's workspace, the network backward's
 * weight-gradient partials and N rows of the privatised levels' input
 * gradient.  SPX_EUNSUPPORTED for configurations the fused path does not
 * cover.
 */
spx_status spx_encode_mlp_bwd_workspace(const spx_encoding* enc, const spx_mlp* mlp, int64_t N, size_t* bytes);

#ifdef __cplusplus
}
#endif

#endif /* SPX_H_ */
