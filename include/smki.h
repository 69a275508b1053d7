/*
 * smki.h -- C ABI of libsmki, an MI355X (gfx950) implementation of the
 * per-scan map update of Bayesian spatial kernel smoothing for dense semantic
 * mapping (S-BKI; Gan, Zhang, Grizzle, Eustice, Ghaffari, arXiv 1909.04631).
 *
 * Conventions for every entry point
 *   - Pointers marked "device" are HIP device pointers (e.g. from a torch
 *     tensor on cuda:N); "host" pointers are read before the call returns.
 *     Arrays of points are row-major float32 [n][3] in metres, 4-byte aligned.
 *   - The caller owns every input and output buffer and keeps it valid until
 *     the map's stream has reached the enqueued work (the same rule as torch).
 *   - A map owns its own device memory (block hash, concentration pool,
 *     scratch); smki_destroy_map frees it.  A map is not thread-safe: use one
 *     host thread and one stream per map.
 *   - No exception or abort crosses the ABI.  Errors detectable on the host
 *     return immediately, enqueue nothing and leave the map unchanged.
 *     Errors found by device validation (bad label, non-finite coordinate,
 *     voxel index outside [-2^20, 2^20), more than 2^20 free samples on one
 *     beam) are detected before any concentration is written, so a failed
 *     insert also leaves the map unchanged.
 *   - Every real parameter is binary32; labels are int32 class ids in
 *     [0, K), or -1 for "drop this hit and its beam".
 */
#ifndef SMKI_H
#define SMKI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t smki_status;
#define SMKI_OK 0
#define SMKI_E_INVALID_ARG (-1)  /* bad pointer, size or parameter (host-checked) */
#define SMKI_E_OOM (-2)          /* device allocation failed */
#define SMKI_E_CAPACITY (-3)     /* a configured limit would be exceeded */
#define SMKI_E_DEVICE (-4)       /* HIP runtime error */
#define SMKI_E_BAD_INPUT (-5)    /* device-detected bad label or non-finite coordinate */
#define SMKI_E_RANGE (-6)        /* voxel index outside [-2^20, 2^20) or beam too long */

typedef struct smki_map smki_map;
typedef struct smki_batch smki_batch;   /* a recorded batched insert (smki_batch_capture) */

/* Map update model (smki_options.model). */
#define SMKI_MODEL_SBKI 0  /* Bayesian spatial kernel inference, Sec. IV, Eq. (7)-(8) */
#define SMKI_MODEL_SCSM 1  /* semantic counting sensor model, Sec. III, Eq. (2): a voxel
                              adds the number of training rows of each class inside it
                              (free-space samples included); exact while a voxel holds
                              fewer than 2^24 rows of a class */

/* Training rows of a voxel (smki_options.selection). */
#define SMKI_SELECT_EXACT 0        /* every row within l: Eq. (7) as written */
#define SMKI_SELECT_FACE_BLOCKS 1  /* rows within l whose block is the voxel's own block or
                                      one of the six sharing a face with it: the extended
                                      block of the paper's implementation (Sec. IV) */

/* Optional settings; pass NULL for defaults (all fields 0). */
typedef struct smki_options {
  int64_t initial_blocks;   /* initial pool capacity in blocks (0: 4096); grows on demand */
  int32_t unit_budget;      /* rows of one (class, block) that one splat work unit
                               takes (0: 512; at most 2^24); a (class, block) holding
                               more rows is split into several units */
  int32_t model;            /* SMKI_MODEL_SBKI (default) or SMKI_MODEL_SCSM; l and sigma0
                               are not used by the counting model */
  int32_t selection;        /* SMKI_SELECT_EXACT (default) or SMKI_SELECT_FACE_BLOCKS
                               (S-BKI only); with face blocks, n_pairs still counts the
                               pairs of the exact support */
  int32_t flags;            /* bit set of SMKI_FLAG_* (0: none) */
} smki_options;

/* smki_options.flags */
#define SMKI_FLAG_WIDE_OFFSETS 1  /* address the partial sums of an insert with 64-bit offsets
                                     even when they take less than 4 GiB (the form used above
                                     4 GiB; results are identical) */

/* Counters of the last insert (smki_last_scan_stats). */
typedef struct smki_scan_stats {
  int64_t n_hits;           /* hit rows: labelled hits kept (label != -1); for soft
                               measurements one per positive class weight */
  int64_t n_free;           /* free-space samples generated */
  int64_t n_point_blocks;   /* map blocks holding at least one training row */
  int64_t n_target_blocks;  /* blocks examined (within reach of a row block) */
  int64_t n_new_blocks;     /* blocks allocated by this insert */
  int64_t n_new_class_blocks; /* class blocks (B^3 concentrations of one class in one
                               block) allocated by this insert; a class no row ever
                               reached in a block takes no memory and reads alpha0 */
  int64_t n_units;          /* splat work units launched */
  int64_t n_updated_voxels; /* voxels with at least one row within l */
  int64_t n_pairs;          /* (voxel, row) pairs with distance < l */
  int64_t n_candidates;     /* (voxel, row) pairs examined: rows x stencil voxels */
  int64_t n_lane_slots;     /* lane-iterations issued (stencil padded to 64-lane steps);
                               n_candidates / n_lane_slots = lane utilisation */
  double splat_ms;          /* device time of the splat kernel (HIP events recorded on
                               the map's stream around its launch) */
  double merge_ms;          /* device time of block allocation and the merge kernel */
} smki_scan_stats;

const char *smki_status_string(smki_status s);

/*
 * Create an empty semantic map (Sec. III-IV of the paper).
 *   res         voxel edge in metres (> 0); voxel (i,j,k) has its centroid at
 *               ((i+1/2) res, (j+1/2) res, (k+1/2) res) -- the query points of
 *               Eq. (7) are the grid centroids (Sec. IV, after Eq. (8)).
 *   block_size  voxels per block edge, a power of two in [1, 32]: the block of
 *               Sec. IV, an octree of grids of depth d holds 2^(d-1) voxels per
 *               edge (depth 1: one voxel).  The counting model serves every
 *               size; S-BKI inserts need B in {2, 4, 8, 16} and a kernel reach
 *               of at most B voxels (else SMKI_E_CAPACITY; see
 *               smki_insert_scan).
 *   l, sigma0   length-scale (> 0) and scale (> 0) of the sparse kernel, Eq. (8).
 *   K           classes (2..255), free class included.
 *   alpha0      Dirichlet prior concentration of every class (> 0), Sec. III.
 *   free_class  class id given to free-space samples, in [0, K).
 * Every voxel of a new map holds alpha0 in every class.
 */
smki_status smki_create_map(float res, int32_t block_size, float l, float sigma0, int32_t K,
                            float alpha0, int32_t free_class, const smki_options *opt,
                            smki_map **out);
smki_status smki_destroy_map(smki_map *m);

/*
 * Per-class kernels: rows of class k use length-scale l[k] and scale
 * sigma0[k] in Eq. (7)-(8), alpha^k = alpha0 + sum_{y_t = k} sigma0[k]
 * f(d / l[k]) (Sec. V-D and VI: the paper keeps both class-independent and
 * names class-dependent values as the way to make them matter).  l and sigma0
 * host float32 [K], each finite and > 0; they apply to later inserts (S-BKI
 * only; the counting model has no kernel).  The stencil follows the largest
 * l[k], so an insert returns SMKI_E_CAPACITY when max l[k] / res >= 4.5.
 * Synchronises the map's stream.  Errors: SMKI_E_INVALID_ARG (map unchanged).
 */
smki_status smki_set_class_params(smki_map *m, const float *l, const float *sigma0);

/*
 * Kernel times of the last inserts, oldest first (synchronises the map's
 * stream): splat_ms[i] the accumulation of Eq. (7)-(8) (HIP events around the
 * splat), merge_ms[i] the allocation of new blocks and the merge into the map.
 * The map keeps the times of its last 64 inserts; *count receives how many
 * were written (at most max).  splat_ms, merge_ms host float32 [max].
 */
smki_status smki_kernel_times(smki_map *m, int32_t max, float *splat_ms, float *merge_ms,
                              int32_t *count);

/*
 * Whether inserts record the HIP events behind smki_kernel_times and the
 * splat / merge times of smki_last_scan_stats (on when a map is created).  Off,
 * an insert enqueues no event (four fewer stream markers per insert); the times
 * then cover only the inserts made while it was on.  No synchronisation.
 * Errors: SMKI_E_INVALID_ARG (m null).
 */
smki_status smki_set_kernel_timing(smki_map *m, int32_t enable);

/* Stream (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream) on which
 * the map enqueues its work; NULL = the default stream. */
smki_status smki_set_stream(smki_map *m, void *hip_stream);

/*
 * Device memory of the map's growable buffers (block hash, block and class-
 * block pools, insert workspaces, recorded batches): alloc(bytes, ctx) returns
 * device memory of the map's device (aligned to at least 256 bytes) or NULL
 * on failure (the call needing it then returns SMKI_E_OOM); release(ptr, ctx)
 * gives back memory alloc returned.  Buffers are released by the allocator
 * that made them, once the map's stream no longer uses them (the map
 * synchronises before it releases).  Both NULL: hipMalloc / hipFree (the
 * default).  Applies to allocations after the call; a few small fixed
 * buffers made at creation always use hipMalloc.  The callbacks run on the
 * thread that calls into the map.  Errors: SMKI_E_INVALID_ARG (exactly one
 * of alloc, release NULL).
 */
typedef void *(*smki_alloc_fn)(size_t bytes, void *ctx);
typedef void (*smki_release_fn)(void *ptr, void *ctx);
smki_status smki_set_allocator(smki_map *m, smki_alloc_fn alloc, smki_release_fn release,
                               void *ctx);

/*
 * Insert one labelled scan: Eq. (7) with the kernel of Eq. (8), applied at
 * every voxel centroid and added to the map (the recursive update of Sec. IV).
 * The training rows are the hits with label != -1 and, for each of them, the
 * free-space samples interpolated along the beam from origin to hit (Sec. III):
 * positions origin + ((j*free_step)/L) * (hit - origin), j = 1..ceil(L/free_step)-1,
 * binary32 arithmetic, labelled free_class.  free_step <= 0: no free samples.
 *   xyz    device float32 [n][3], label device int32 [n], origin host float32 [3].
 * Returns after the work is enqueued (it synchronises the stream internally
 * to size its launches).  Errors: SMKI_E_BAD_INPUT for a label outside
 * {-1..K-1} or a non-finite kept coordinate, SMKI_E_RANGE for a voxel index
 * outside [-2^20, 2^20) or a beam with more than 2^20 samples, SMKI_E_CAPACITY
 * when the kernel's reach R (the voxels a row's support extends past its own
 * voxel: R = ceil(l / res + 1/2) - 1, at most 4, so l / res < 4.5) exceeds 4 or
 * the block size B, when B is not 2, 4, 8 or 16 (S-BKI), or when the scan's
 * bounding box spans more than 2^30 / K blocks; on any error the map is left
 * unchanged.
 */
smki_status smki_insert_scan(smki_map *m, const float *xyz, const int32_t *label, int64_t n,
                             const float *origin, float free_step);

/*
 * Insert one scan of soft measurements (Sec. VI: a classifier's pseudo-
 * probability vector per hit instead of one label).  probs device float32
 * [n][K], row i the class weights of hit i, each finite and >= 0.  Every
 * class k with probs[i][k] > 0 adds probs[i][k] * sigma0 f(d / l) to its
 * concentration at every voxel centroid within l (S-BKI), or probs[i][k] to
 * the hit's own voxel (S-CSM) -- the linear-pooling form; the weights are
 * used as given, without renormalisation, so a one-hot row is the
 * smki_insert_scan update.  A row of zeros drops the hit and its beam (as
 * label -1); the free-space samples of the other beams are free_class rows of
 * weight 1.  xyz, origin, free_step and the errors are those of
 * smki_insert_scan (a negative or non-finite weight: SMKI_E_BAD_INPUT), plus
 * SMKI_E_CAPACITY when n * K > 2^30.  The scan statistics count one hit row
 * per positive weight.
 */
smki_status smki_insert_scan_soft(smki_map *m, const float *xyz, const float *probs, int64_t n,
                                  const float *origin, float free_step);

/*
 * Insert S scans in one pass: rows offsets[s]..offsets[s+1]-1 of xyz/label
 * belong to scan s, whose beams start at origins[s].  Eq. (7) is additive over
 * training rows, so the result equals S sequential inserts up to float32
 * summation order.  offsets host int64 [S+1] (offsets[0] = 0, non-decreasing),
 * origins host float32 [S][3].
 */
smki_status smki_insert_scans(smki_map *m, const float *xyz, const int32_t *label,
                              const int64_t *offsets, const float *origins, int32_t S,
                              float free_step);

/*
 * Batched insert recorded as one HIP graph and replayed without any host
 * synchronisation (Eq. (7) is additive over training rows, Sec. IV's recursive
 * update, so S scans go in one pass as in smki_insert_scans).
 *
 * smki_batch_capture performs smki_insert_scans(m, xyz, label, offsets,
 * origins, S, free_step) -- an ordinary insert, which updates the map and
 * synchronises -- and then records the same insert for the same device buffers
 * xyz / label, the same n = offsets[S], S and free_step into a graph in which
 * every launch reads its counts from device memory.  Capacities are that
 * insert's sizes grown by `margin` (0..16, e.g. 0.25): training rows, work
 * units, the voxel box (grown by margin of its extent on every side), and room
 * in the map's pools for that insert's new blocks once more.  S-BKI maps only.
 *
 * smki_batch_replay launches the graph on the map's stream: the insert of what
 * xyz / label hold at the time it runs, with these scan offsets (host int64
 * [S+1], offsets[S] = the captured n) and origins (host float32 [S][3]).  It
 * returns once the graph is enqueued (it waits only for the previous replay of
 * the same batch to finish).  A replay whose data needs more than the captured
 * capacities, or whose rows leave the captured voxel box, writes nothing to
 * the map; its error (SMKI_E_CAPACITY, SMKI_E_RANGE, SMKI_E_BAD_INPUT) is
 * reported by the next smki_sync.  A replay returns SMKI_E_CAPACITY at once
 * when the map's storage moved since the capture (an ordinary insert or an
 * import grew it; smki_set_class_params also invalidates the recording):
 * capture again.  smki_last_scan_stats reports the replay's counters (times
 * are not recorded).  Destroy batches before their map.
 */
smki_status smki_batch_capture(smki_map *m, const float *xyz, const int32_t *label,
                               const int64_t *offsets, const float *origins, int32_t S,
                               float free_step, float margin, smki_batch **out);
smki_status smki_batch_replay(smki_batch *b, const int64_t *offsets, const float *origins);
smki_status smki_batch_destroy(smki_batch *b);

/*
 * Read voxels (Sec. III, Eq. (3)-(4), reused for S-BKI in Sec. IV):
 *   ijk    device int32 [M][3] voxel indices;
 *   alpha  device float32 [M][K]  concentrations (nullable);
 *   mean   device float32 [M][K]  alpha / sum(alpha)                (nullable);
 *   var    device float32 [M][K]  mean (1 - mean) / (sum(alpha)+1)  (nullable);
 *   label  device int32 [M]       argmax of alpha, lowest index on ties (nullable);
 *   p_occ  device float32 [M]     1 - mean of the free class (nullable).
 * Voxels never updated read alpha0 in every class.
 */
smki_status smki_query(smki_map *m, const int32_t *ijk, int64_t M, float *alpha, float *mean,
                       float *var, int32_t *label, float *p_occ);

/* Number of allocated blocks. */
smki_status smki_num_blocks(smki_map *m, int64_t *n_blocks);

/*
 * Checkpoint: *n_blocks (host) receives the number of blocks.  If block_ijk
 * and alpha are non-NULL and capacity >= *n_blocks, writes the blocks in
 * ascending key order: block_ijk device int32 [n][3] (block coordinates:
 * voxel index >> log2(block_size)), alpha device float32 [n][K][B^3]
 * (class-major; voxel (x,y,z) of a block at (x*B + y)*B + z).
 */
smki_status smki_export(smki_map *m, int64_t capacity, int64_t *n_blocks, int32_t *block_ijk,
                        float *alpha);
/* Replace the map's contents with n exported blocks (device arrays as above;
 * block i of the input becomes the map's block i).  n = 0 empties the map
 * (capacity is kept) without synchronising the stream; n > 0 validates the
 * input on the device and synchronises once to read the result and size the
 * class blocks.  Errors: SMKI_E_RANGE if a block's voxels leave
 * [-2^20, 2^20), SMKI_E_BAD_INPUT if a block appears twice, SMKI_E_CAPACITY
 * if n * K > 2^30, SMKI_E_OOM; on any error the map is left unchanged. */
smki_status smki_import(smki_map *m, int64_t n, const int32_t *block_ijk, const float *alpha);

/* The counters of the last insert or replay (smki_scan_stats).  They stay on
 * the device until asked for: the first call after an insert synchronises the
 * map's stream and reads them back.  Errors: SMKI_E_INVALID_ARG. */
smki_status smki_last_scan_stats(smki_map *m, smki_scan_stats *out);

/* Wait for the map's stream; returns a deferred device error if one occurred. */
smki_status smki_sync(smki_map *m);

/*
 * The free-space samples of one scan alone (Sec. III; same binary32 recipe as
 * the insert).  Two calls: with out_xyz == NULL only *n_out (host) is set;
 * then out_xyz device float32 [n_out][3] and out_parent device int64 [n_out]
 * (nullable; index of the source hit) are filled in (hit, j) order.
 *   K is used to validate the labels.  Synchronous on hip_stream.
 */
smki_status smki_free_samples(const float *xyz, const int32_t *label, int64_t n, const float *origin,
                              float free_step, int32_t K, void *hip_stream, int64_t *n_out,
                              float *out_xyz, int64_t *out_parent);

/*
 * The voxel-cell table of a set of rows (the bucketing step of the update):
 * rows are keyed by voxel index floor(x / res) (binary32 division) and radix
 * sorted.  Two calls: with cell_keys == NULL only *n_cells (host) is set; then
 *   cell_keys  device uint64 [n_cells] packed voxel index
 *              ((i + 2^20) << 42) | ((j + 2^20) << 21) | (k + 2^20),
 *   cell_start device int32 [n_cells], cell_count device int32 [n_cells],
 *   order      device int32 [n] (nullable): row ids in sorted order, so rows
 *              order[cell_start[c] .. cell_start[c]+cell_count[c]-1] are cell c's.
 * Cells appear in the library's sort order (block-major).  Synchronous.
 */
smki_status smki_bucket_cells(const float *xyz, int64_t n, float res, int32_t block_size,
                              void *hip_stream, int64_t *n_cells, uint64_t *cell_keys,
                              int32_t *cell_start, int32_t *cell_count, int32_t *order);

/*
 * Differentiable form (an extension; the paper tunes l and sigma0 by hand and
 * names hyper-parameter optimisation as future work, Sec. VI).  Stateless:
 * explicit training rows (hits and free samples) and labelled query points.
 *   alpha_q[h][k] = alpha0 + sum_t sigma0 f(|x_t - x_h| / l) [y_t = k]   (Eq. (7)-(8))
 *   loss = -(1/H) sum_h log(alpha_q[h][y_h] / sum_k alpha_q[h][k])
 *   train_xyz device float32 [n_train][3], train_label device int32 [n_train],
 *   query_xyz device float32 [n_query][3], query_label device int32 [n_query],
 *   loss device float32 [1]; alpha_q device float32 [n_query][K] (nullable).
 * workspace: device scratch of smki_loss_workspace_bytes(...) bytes, or NULL to
 * let the call allocate its own.
 */
size_t smki_loss_workspace_bytes(int64_t n_train, int64_t n_query, int32_t K);
smki_status smki_loss_forward(const float *train_xyz, const int32_t *train_label, int64_t n_train,
                              const float *query_xyz, const int32_t *query_label, int64_t n_query,
                              float l, float sigma0, float alpha0, int32_t K, void *hip_stream,
                              void *workspace, size_t workspace_bytes, float *loss,
                              float *alpha_q);
/*
 * Gradient of loss * grad_loss (grad_loss device float32 [1]) with respect to
 * l, sigma0 (device float32 [1] each, nullable), the training coordinates
 * (device float32 [n_train][3], nullable) and the query coordinates (device
 * float32 [n_query][3], nullable).  alpha_q is the forward's output.  Kernel
 * weights are recomputed, not stored.
 */
smki_status smki_loss_backward(const float *train_xyz, const int32_t *train_label, int64_t n_train,
                               const float *query_xyz, const int32_t *query_label, int64_t n_query,
                               float l, float sigma0, float alpha0, int32_t K, void *hip_stream,
                               void *workspace, size_t workspace_bytes, const float *alpha_q,
                               const float *grad_loss, float *grad_l, float *grad_sigma0,
                               float *grad_train_xyz, float *grad_query_xyz);

/*
 * The same loss with per-class kernels (the class-dependent l and sigma0 that
 * Sec. V-D and VI point to):  alpha_q[h][k] = alpha0 + sum_{t: y_t = k}
 * sigma0[k] f(|x_t - x_h| / l[k]).  l, sigma0 host float32 [K], each finite and
 * > 0.  Other arguments as smki_loss_forward; the workspace size is
 * smki_loss_workspace_bytes(n_train, n_query, K).
 */
smki_status smki_loss_forward_classes(const float *train_xyz, const int32_t *train_label,
                                      int64_t n_train, const float *query_xyz,
                                      const int32_t *query_label, int64_t n_query, const float *l,
                                      const float *sigma0, float alpha0, int32_t K,
                                      void *hip_stream, void *workspace, size_t workspace_bytes,
                                      float *loss, float *alpha_q);
/*
 * Its gradient: grad_l and grad_sigma0 device float32 [K] (nullable) receive
 * dloss/dl[k] and dloss/dsigma0[k]; coordinates as smki_loss_backward.  The
 * per-class gradients are summed over queries in double, in a fixed order.
 */
smki_status smki_loss_backward_classes(const float *train_xyz, const int32_t *train_label,
                                       int64_t n_train, const float *query_xyz,
                                       const int32_t *query_label, int64_t n_query,
                                       const float *l, const float *sigma0, float alpha0,
                                       int32_t K, void *hip_stream, void *workspace,
                                       size_t workspace_bytes, const float *alpha_q,
                                       const float *grad_loss, float *grad_l, float *grad_sigma0,
                                       float *grad_train_xyz, float *grad_query_xyz);

/*
 * smki_loss_forward without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Arguments and results are those of
 * smki_loss_forward; the workspace is a fixed device array inside the library
 * (SMKI_LOSS_NOALLOC_BYTES, 64 MiB; each device the library runs on holds its
 * own copy until the process ends), so the call allocates nothing.  The
 * device current at the call must be the device of hip_stream.  Inputs whose
 * workspace would exceed SMKI_LOSS_NOALLOC_BYTES return SMKI_E_CAPACITY
 * (roughly above 5e5 training rows, or a sparse set spanning a large box).
 * Every call on one device shares that device's array: calls that overlap on
 * one device (several host threads or streams) race and must be serialised
 * by the caller.  Synchronises hip_stream once (to size the grid), like
 * smki_loss_forward.
 */
#define SMKI_LOSS_NOALLOC_BYTES ((size_t)64 << 20)
smki_status smki_loss_forward_noalloc(const float *train_xyz, const int32_t *train_label,
                                      int64_t n_train, const float *query_xyz,
                                      const int32_t *query_label, int64_t n_query, float l,
                                      float sigma0, float alpha0, int32_t K, void *hip_stream,
                                      float *loss, float *alpha_q);

#ifdef __cplusplus
}
#endif
#endif /* SMKI_H */
