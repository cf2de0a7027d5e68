/*
 * si.h -- C ABI of the MI355X (gfx950) spin-image library.
 *
 * Computes spin images (Section 2.1, Algorithm 1 of "Efficient Generation of
 * Parallel Spin-images Using Dynamic Loop Scheduling", arXiv 1811.00901):
 * for every chosen oriented point P = (p, n) and every scene point X = (x, n_x)
 *
 *     beta  = n . (x - p)
 *     alpha = sqrt(|x - p|^2 - beta^2)
 *
 * X is rejected when the angle between n and n_x exceeds the support angle S
 * or when its bin falls outside the W x W image; otherwise it is accumulated
 * into P's image.  The per-image loop is a DOALL loop (Section 2.2) that the
 * library distributes over persistent GPU workgroups with the loop-scheduling
 * techniques of Section 2.2 (STATIC, SS, GSS, FAC) or with an order and chunk
 * sizes predicted by a learned per-image cost model.
 *
 * Conventions for every entry point:
 *   - All functions return si_status and never abort or throw across the ABI;
 *     si_last_error() gives a thread-local text for the last failure.
 *   - "device" pointers are HIP device memory on the current device (for
 *     example the storage of a torch tensor); "host" pointers are CPU memory.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued asynchronously on it; input and output buffers must stay valid
 *     until the stream has reached the call.  Where a function must read a
 *     result back to the host it synchronises the stream, and says so.
 *   - The caller owns every buffer it passes in.  The library owns scenes and
 *     cost models until the matching si_free_* call.
 *   - Chunk tables are built on the host once per schedule and device, then
 *     uploaded on the stream of their first use (from pinned staging, without
 *     waiting) and cached (64 per device; the least recently used is freed
 *     once the launches that read it are done).
 *   - si_build_scene(s), si_generate, si_generate_batched, si_autotune and
 *     si_generate_noalloc upload host data or wait on the host, so they
 *     cannot be captured into a graph: on a capturing hip_stream they return
 *     SI_E_UNSUPPORTED before enqueuing anything.  si_generate_batched with
 *     use_graph = 1 captures and replays a graph of its own instead.
 *   - Distinct scenes, models and streams may be used from different threads.
 *     Calls that run concurrently on different streams share a pool of 64
 *     work-counter slots per device, so at most 64 generation launches may be
 *     in flight at once.
 */
#ifndef SI_H
#define SI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SI_ABI_VERSION 1

typedef enum si_status {
    SI_OK = 0,
    SI_E_INVALID = -1,     /* an argument is out of its documented domain */
    SI_E_OOM = -2,         /* device or host allocation failed */
    SI_E_DEVICE = -3,      /* a HIP runtime call failed */
    SI_E_UNSUPPORTED = -4  /* valid request the library does not implement */
} si_status;

/* Loop-scheduling techniques (Section 2.2) plus the learned schedule. */
enum {
    SI_SCHED_STATIC = 0,  /* one contiguous block per workgroup, no counter   */
    SI_SCHED_SS = 1,      /* self-scheduling: one image per claim             */
    SI_SCHED_GSS = 2,     /* guided: ceil(remaining / P) per claim            */
    SI_SCHED_FAC = 3,     /* factoring: batches of P chunks ceil(R_b/(x P))   */
    SI_SCHED_LEARNED = 4, /* cost-model order + cost-weighted factoring       */
    /* two later techniques of the family (the paper's future work) */
    SI_SCHED_TSS = 5,     /* trapezoid: sizes fall linearly from N/(2P) to 1  */
    SI_SCHED_FAC_PROB = 6,/* probabilistic factoring from the cost's sigma/mu */
    /* three whose chunk depends on the requesting workgroup, sized when it
       claims (si_generate only; see si_sched) */
    SI_SCHED_WF = 7,      /* weighted factoring: FAC2 batches x worker weight */
    SI_SCHED_AWF = 8,     /* adaptive weighted factoring: weights measured    */
    SI_SCHED_AF = 9       /* adaptive factoring: from measured mu, sigma      */
};

/* Binning of a pair into the image (see si_params). */
enum {
    SI_BIN_BILINEAR = 0,
    SI_BIN_CEIL = 1
};

typedef struct si_scene si_scene;           /* opaque, library-owned */
typedef struct si_cost_model si_cost_model; /* opaque, library-owned */

/*
 * Spin-image parameters (Section 2.1 and the notation table): W pixels per
 * side, bin size B in scene units, support angle S in radians.
 *   W    in [2, 64]
 *   bin  finite, > 0
 *   support_angle finite, >= 0; values >= pi disable the angle test (the
 *        paper's runs use S = 2 pi, Section 4.1).  The test acos(n.n_x) <= S
 *        is evaluated as n.n_x >= cos(S) with cos(S) computed in double
 *        precision and rounded to float.
 *   mode SI_BIN_CEIL: the printed binning, k = ceil(W/2 - beta/B) (row),
 *        l = ceil(alpha/B) (column), counted when 0 <= k, l < W, bin += 1.
 *        SI_BIN_BILINEAR: with v = W/2 - beta/B and u = alpha/B, a unit
 *        weight spread over the four grid nodes around (v, u); counted when
 *        0 <= v < W-1 and u < W-1.  Weights are accumulated as exact 16.16
 *        fixed point (each pair adds exactly 1.0 to the image), so images do
 *        not depend on summation order.
 */
typedef struct si_params {
    int32_t W;
    float bin;
    float support_angle;
    int32_t mode;
} si_params;

/*
 * Schedule of the per-image loop over P persistent workgroups.
 *   kind            SI_SCHED_*
 *   num_workgroups  P; 0 = library default for the device and W
 *   min_chunk       lower bound of every dynamic chunk (0 or 1 = none;
 *                   0 in a batched SI_SCHED_FAC launch over several scenes
 *                   takes 16)
 *   fac_divisor     x of SI_SCHED_FAC / SI_SCHED_LEARNED; 0 = 2 (FAC2), except
 *                   that a batched SI_SCHED_FAC launch over several scenes
 *                   takes 12 (their concatenated loop's iteration costs vary
 *                   far more than one scene's, and the batch ratio grows
 *                   with that variation; smaller first batches also keep
 *                   the workgroups running at once on fewer scenes).
 *                   For SI_SCHED_FAC_PROB: cv = sigma / mu of the per-image
 *                   cost (>= 0), which sets each batch's ratio x_j
 *                   (Hummel, Schonberg and Flynn 1992): with
 *                   b_j = P cv / (2 sqrt(R_j)), x_0 = 1 + b_0^2 +
 *                   b_0 sqrt(b_0^2 + 2), x_j = 2 + b_j^2 + b_j sqrt(b_j^2 + 4);
 *                   cv = 0 gives one batch (STATIC's blocks, claimed
 *                   dynamically).  SI_SCHED_TSS (Tzen and Ni 1993): chunk i
 *                   has ceil(F - i delta) iterations, F = ceil(N / (2P)),
 *                   delta = (F - L) / (C - 1) (real), C = ceil(2N / (F + L)),
 *                   never below L = max(1, min_chunk).
 *                   SI_SCHED_WF, SI_SCHED_AWF, SI_SCHED_AF size each chunk
 *                   when a workgroup claims it (a claim counter gives its
 *                   batch, an atomic addition of the size its start):
 *                   WF (Hummel, Schmidt, Uma and Wein 1996): claim r is in
 *                   batch b = r / P, whose FAC2 chunk c_b (divisor x, as
 *                   for FAC) is scaled by the workgroup's weight w
 *                   (si_set_worker_weights; else the emulated speeds of
 *                   si_set_emulated_workers; else 1), weights scaled to sum
 *                   P: ceil(w c_b) iterations.  AWF (Banicescu, Velusamy and
 *                   Devaprasad 2003, adapting after every chunk): WF with
 *                   w_i = P r_i / sum_j r_j, r_i = sum_k k n_ik / sum_k k t_ik
 *                   over workgroup i's completed chunks (the sum over the
 *                   measured workgroups, scaled by P over their number; 1
 *                   before a first chunk).  AF (Banicescu and Liu 2000):
 *                   (D + 2TR - sqrt(D^2 + 4DTR)) / (2 mu_i) iterations for R
 *                   left, D = sum sigma_j^2 / mu_j, T = 1 / sum 1 / mu_j, mu
 *                   and sigma the mean and deviation of each workgroup's
 *                   time per image (sampled per group of images; sums over
 *                   the measured workgroups scaled to P); a first claim gets
 *                   FAC2's first chunk.  Chunk sizes of these three depend
 *                   on timing; images never do.  For these three,
 *                   min_chunk 0 means 8 (one unit of the spread order:
 *                   smaller chunks cannot share candidate passes between
 *                   images).  They run in si_generate only
 *                   (SI_E_UNSUPPORTED elsewhere).
 *   model           SI_SCHED_LEARNED only; trained cost model
 *   fallback_to_fac SI_SCHED_LEARNED without a model: 1 = run FAC, 0 = error
 *   group           images that share one pass over their common candidate
 *                   points (1..8); 0 = library default
 *   order           SI_ORDER_SPREAD (0): the oriented points sorted by their
 *                   place in the scene (grid cell, then quarter of the cell
 *                   along x), in units of 8 consecutive iterations, and the
 *                   units taken with a stride coprime to their number, so
 *                   that every part of the loop holds units from the whole
 *                   scene (chunks of neighbouring images keep sharing
 *                   candidates, while costs stop clustering along the loop;
 *                   SI_SCHED_LEARNED builds its own order from the sorted
 *                   one); SI_ORDER_CELL (2): the loop runs over the oriented
 *                   points in that sorted order, so that neighbouring images share
 *                   candidates (iterations of a DOALL loop may run in any
 *                   order); SI_ORDER_GIVEN (1): in the order of oriented_idx,
 *                   as the paper's loop i = 0..N-1.  Chunks are contiguous
 *                   ranges of that order.  Images are the same either way.
 */
typedef struct si_sched {
    int32_t kind;
    int32_t num_workgroups;
    int32_t min_chunk;
    float fac_divisor;
    const si_cost_model* model;
    int32_t fallback_to_fac;
    int32_t group;
    int32_t order;
} si_sched;

enum {
    SI_ORDER_SPREAD = 0,
    SI_ORDER_GIVEN = 1,
    SI_ORDER_CELL = 2
};

/*
 * Optional run statistics, filled after synchronising the stream.
 *   kernel_ms        device time of the generation launch(es) (HIP events)
 *   pairs_in_support sum of the per-image in-support counts
 *   pairs_tested     candidate pairs evaluated (after cell-list pruning)
 *   sched_used       the SI_SCHED_* actually run (FAC when LEARNED fell back)
 *   n_wg, n_chunks   workgroups launched, chunks in the schedule
 *   n_invalid        oriented indices outside [0, M) (their images are zero
 *                    and their count is 0xFFFFFFFF; the call returns
 *                    SI_E_INVALID when this is nonzero)
 *   n_overflow       images re-accumulated on the 64-bit path because an
 *                    image had 65536 or more in-support pairs
 *   wg_busy_ns       caller-owned host array of wg_busy_cap entries or NULL;
 *                    receives each workgroup's busy time in ns
 */
typedef struct si_stats {
    double kernel_ms;
    uint64_t pairs_in_support;
    uint64_t pairs_tested;
    int32_t sched_used;
    int32_t n_wg;
    int32_t n_chunks;
    int32_t n_invalid;
    int32_t n_overflow;
    int32_t wg_busy_cap;
    uint64_t* wg_busy_ns;
} si_stats;

/* Static facts about a built scene. */
typedef struct si_scene_info {
    int64_t M;
    float cell_size;            /* edge of a grid cell (scene units) */
    float max_support_radius;   /* largest support radius the grid is valid for */
    int32_t dims[3];            /* cells per axis */
    float origin[3];            /* lower corner of the grid */
    int64_t n_cells;
} si_scene_info;

/*
 * Build a scene: the list of oriented points OP (Section 2.1) in the layout
 * the kernels read -- a uniform grid of cells of edge h >= R / 3 (three cells
 * per support radius), points sorted by cell, and within a cell by the quarter
 * of the cell their x falls in, into 32-byte float4 position and normal
 * records.  The grid is conservative for every pair with
 * |x - p| <= max_support_radius; max_support_radius <= 0 builds a single
 * cell (brute force over all M points, the paper's O(N M) loop).
 *   points_xyz, normals_xyz  device, M x 3 float32, row-major; read only
 *   M                        number of oriented points, > 0, < 2^31
 * Synchronises the stream once (to read the bounding box); the rest of the
 * build is queued on hip_stream, so the scene is ready for work queued after
 * it on that stream (other streams must wait for it, e.g. on an event).  The
 * scene's device arrays come from the device's stream-ordered memory pool.
 * Returns SI_E_INVALID for M <= 0, NULL pointers or a non-finite radius; a
 * NaN coordinate is placed in cell 0 and is never in support of anything.
 */
si_status si_build_scene(const float* points_xyz, const float* normals_xyz, int64_t M,
                         float max_support_radius, void* hip_stream, si_scene** out);

/* One scene of si_build_scenes: the arguments of si_build_scene. */
typedef struct si_scene_desc {
    const float* points_xyz;    /* device, M x 3 float32; read only */
    const float* normals_xyz;   /* device, M x 3 float32; read only */
    int64_t M;                  /* > 0, < 2^31 */
    float max_support_radius;   /* as for si_build_scene */
} si_scene_desc;

/*
 * Build n scenes at once (for batches of many scenes, si_generate_batched):
 * each out[i] is the scene si_build_scene builds from descs[i] -- the same
 * grid and the same points in every cell key; points of one key may lie in
 * another order, which no image, count or feature depends on.  The work is
 * a fixed number of launches for all scenes together (bounding boxes, then
 * binning, scan and scatter in sub-batches of at most 2^27 cell keys and
 * 2^28 points, any single scene accepted), with one synchronisation for the
 * bounding boxes and one per sub-batch, instead of one synchronisation and
 * about ten launches per scene.  On return every out[i] is ready for work on
 * any stream.  The scenes' arrays share one allocation from the device's
 * pool, released with the last of them; each scene is released with
 * si_free_scene, in any order (the others stay valid).
 *   descs  host array of n descriptions; out  host array of n handles
 * n == 0 does nothing.  Returns SI_E_INVALID (naming the scene) for an
 * invalid description, NULL descs/out or n < 0; on any error no scene is
 * built and every out[i] is NULL.
 */
si_status si_build_scenes(const si_scene_desc* descs, int32_t n, void* hip_stream,
                          si_scene** out);

/* Release a scene (NULL is ignored).  Work using it must have completed. */
void si_free_scene(si_scene* scene);

/* Fill *out with the scene's grid description (host). */
si_status si_scene_info_get(const si_scene* scene, si_scene_info* out);

/*
 * Largest |x - p| of a pair that can be inside the image for these params
 * (closed form of the extent conditions), written to *radius (host).
 */
si_status si_support_radius(const si_params* params, float* radius);

/*
 * Generate N spin images (Section 2.1, Algorithm 1; each claimed chunk
 * [start, end) is Algorithm 2).
 *   oriented_idx  device, N int32 indices into the scene's points in the
 *                 order given to si_build_scene; duplicates allowed.  The
 *                 paper's case is 0..N-1.
 *   images_out    device, N x W x W float32; image i (of oriented_idx[i]) is
 *                 images_out[i], row index = beta axis, column = alpha axis
 *   counts_out    device, N uint32 in-support counts
 *   stats         host or NULL; when set the stream is synchronised
 * The images and counts do not depend on the schedule or on thread timing.
 * Returns SI_E_INVALID for bad params/schedule, a support radius above the
 * scene's max_support_radius, or (when stats is set) invalid indices.  An
 * index outside [0, M) is found on the device: its image is zero, its count
 * 0xFFFFFFFF, and the device's invalid-index flag is set, which
 * si_device_errors reports (the call itself returns before the launch has
 * run, so without stats it cannot).
 * N == 0 is a no-op returning SI_OK.
 */
si_status si_generate(const si_scene* scene, const int32_t* oriented_idx, int64_t N,
                      const si_params* params, const si_sched* sched,
                      float* images_out, uint32_t* counts_out, si_stats* stats,
                      void* hip_stream);

/* One scene's share of a batched launch. */
typedef struct si_batch_item {
    const si_scene* scene;
    const int32_t* oriented_idx;  /* device */
    int64_t N;
    si_params params;
    float* images_out;            /* device, N x W x W */
    uint32_t* counts_out;         /* device, N */
} si_batch_item;

/*
 * Generate the images of many scenes in one persistent launch per image-size
 * class: one flattened schedule whose chunks never span two scenes.  Items
 * with W <= 32 and with W > 32 form two classes, launched one after the other
 * on the stream, each with its own schedule and its own default group and
 * workgroup count (a launch sizes its LDS for its largest image, so small
 * images next to W = 64 ones would run at a lower occupancy); sched applies
 * to both.  use_graph = 1 captures the launches in one HIP graph that is
 * cached and replayed while the item list (pointers, sizes, params) and
 * schedule are unchanged.  In the statistics, n_wg and wg_busy_ns are those
 * of the larger launch's workgroup slots, busy times summed over the
 * launches; kernel_ms runs from the first spin launch to the end of the last.  sched->kind is any
 * SI_SCHED_*.  SI_SCHED_LEARNED plans the whole batch on the device before
 * the launch (inside the graph): features and predicted costs of every
 * image, units of 16 iterations that never cross an item, one
 * longest-first order of all units, factoring on predicted cost into
 * chunks, and each chunk split into its runs of one item; at most 4,096
 * workgroups, as in si_generate.  Every item is validated as in si_generate; results are identical to one si_generate per
 * item.  Items with N == 0 are skipped.  Without a graph the call stages its
 * tables and synchronises the stream once before launching; the first call
 * with a new item list in graph mode also synchronises (capture).  The graph
 * cache holds up to 8 item lists per process.  An entry is keyed on the
 * scenes' and cost model's identities (serial numbers that are never reused,
 * not their addresses) and on the index and output pointers; it holds those
 * buffers' device pointers, so a replay needs them alive.  si_free_scene and
 * si_free_cost_model drop every entry built for the freed object, so a scene
 * or model created later at the same address gets a graph of its own.
 */
si_status si_generate_batched(const si_batch_item* items, int32_t n_items,
                              const si_sched* sched, int32_t use_graph,
                              si_stats* stats, void* hip_stream);

/*
 * Autotuner: picks the launch parameters of a workload (the items as for
 * si_generate_batched; one item for a single scene) for scheduling technique
 * `kind`.  Tuned: group (images per shared candidate pass, from 1, 2, 4, 6,
 * 8), num_workgroups (2, 3, 4, 5, 6 or 8 per compute unit), fac_divisor (FAC and
 * LEARNED: 1.5, 2, 3, 4, 8, 12, 16), min_chunk (dynamic techniques: 0, 4, 16)
 * and, jointly with chunk sizes, the loop order (dynamic techniques other
 * than LEARNED: order, min_chunk and, for FAC, fac_divisor set together to
 * cell 32 x16, cell 32 x64, cell 16 x16 or spread 16 x12; small chunks over
 * the cell order make every workgroup sweep the scene at once, which keeps
 * the groups running together on shared candidates), by two sweeps of
 * coordinate descent from the library's defaults (group and num_workgroups
 * 0: chosen per launch; a tuned value applies to every launch),
 * at most max_trials timed candidates (each the median of two launches after
 * a warm-up).  Every candidate's images and counts must give the same 64-bit
 * checksum as the first one, else SI_E_DEVICE.  The winner is written to
 * *best (kind filled, model NULL) and its time to *best_ms (host, may be
 * NULL).  Winners are cached per (device, kind, use_graph, image widths, size class) in memory
 * and, when the environment variable SI_AUTOTUNE_CACHE names a file, in that
 * file (one JSON object per line; unreadable lines are ignored).  A cached
 * winner is returned without running unless force = 1.  The items' output
 * buffers are overwritten.  Synchronises the stream.
 */
si_status si_autotune(const si_batch_item* items, int32_t n_items, int32_t kind,
                      int32_t use_graph, int32_t max_trials, int32_t force, si_sched* best,
                      double* best_ms, void* hip_stream);

/*
 * Per-image cost features (12 float32 per image, device N x 12) of the
 * oriented points, from the occupancy of the 3 x 3 x 3 block of cells of size
 * close to the support radius around p and from n.  Used by the learned cost
 * model; not part of any image.
 */
si_status si_features(const si_scene* scene, const int32_t* oriented_idx, int64_t N,
                      const si_params* params, float* feats_out, void* hip_stream);

/*
 * The same features for many scenes at once, as the batched learned
 * schedule computes them: feats_out (device) receives sum(N) x 12 floats,
 * the items' rows one after the other in item order (items with N == 0 add
 * none).  The items' output buffers are not used.  Synchronises the stream.
 */
si_status si_features_batched(const si_batch_item* items, int32_t n_items, float* feats_out,
                              void* hip_stream);

/*
 * Learned per-image cost model: an MLP 12 -> 64 -> 64 -> 1 (ReLU, float32)
 * predicting log(1 + in-support count) from the features above.
 */
si_status si_cost_model_create(uint64_t seed, si_cost_model** out);
void si_free_cost_model(si_cost_model* model);

/*
 * Train with Adam (beta1 0.9, beta2 0.999, eps 1e-8) on mean squared error
 * against log1p(counts), on the device.
 *   feats   device n x 12 float32; counts device n uint32
 *   epochs  passes over the data; batch: minibatch size (1..65536)
 *   loss_curve_host  host array of `epochs` floats (mean loss per epoch) or
 *                    NULL; when set the stream is synchronised
 * Minibatches are contiguous slices of a per-epoch permutation drawn from the
 * model's seed.
 */
si_status si_cost_model_train(si_cost_model* model, const float* feats, const uint32_t* counts,
                              int64_t n, int32_t epochs, float lr, int32_t batch,
                              float* loss_curve_host, void* hip_stream);

/*
 * Gradient of the mean squared error over all n samples with respect to the
 * 5,057 parameters (layout as in si_cost_model_get_params), computed on the
 * device with the training kernels, copied to grad_host (host, 5,057
 * floats); the loss to *loss_host (may be NULL).  Does not change the model.
 * Synchronises the stream.
 */
si_status si_cost_model_gradient(const si_cost_model* model, const float* feats,
                                 const uint32_t* counts, int64_t n, float* grad_host,
                                 float* loss_host, void* hip_stream);

/* Predicted in-support counts (expm1 of the network output), device n floats. */
si_status si_cost_model_predict(const si_cost_model* model, const float* feats, int64_t n,
                                float* pred_counts, void* hip_stream);

/*
 * The same predictions as the learned schedule's planner computes them:
 * fp16 operands and fp32 accumulation on the matrix cores (features,
 * weights and hidden activations rounded to fp16; biases, sums and the
 * output in fp32).  The planner only groups predicted unit costs into 32
 * buckets per octave, far coarser than this rounding.  Arguments as for
 * si_cost_model_predict; feats must be 16-byte aligned (SI_E_INVALID
 * otherwise).
 */
si_status si_cost_model_predict_planner(const si_cost_model* model, const float* feats, int64_t n,
                                        float* pred_counts, void* hip_stream);

/* Copy the 5,057 parameters (W1 64x12, b1 64, W2 64x64, b2 64, w3 64, b3 1, in
 * that order, row-major) between the model and a host array. */
si_status si_cost_model_get_params(const si_cost_model* model, float* host_params, int64_t n);
si_status si_cost_model_set_params(si_cost_model* model, const float* host_params, int64_t n);

/* Save / load the parameters to a file (little-endian header + float32). */
si_status si_cost_model_save(const si_cost_model* model, const char* path);
si_status si_cost_model_load(const char* path, si_cost_model** out);

/*
 * Host-only: the chunk table the generation launch uses for a schedule.
 * Writes chunk starts (n_chunks + 1 entries, the last = N) to starts_out
 * (host, capacity cap) and the count to *n_chunks.  STATIC gives P
 * balanced blocks; SS, GSS and FAC follow Section 2.2 (FAC as FAC2 with
 * divisor x); SI_SCHED_TSS and SI_SCHED_FAC_PROB as in si_sched (for
 * FAC_PROB, fac_divisor carries sigma / mu).  SI_SCHED_LEARNED has no
 * fixed table (si_learned_table).  Returns SI_E_INVALID when cap is too
 * small or the kind is unknown.
 */
si_status si_chunk_table(int32_t kind, int64_t N, int32_t P, int32_t min_chunk,
                         float fac_divisor, int64_t* starts_out, int64_t cap,
                         int64_t* n_chunks);

/*
 * Host-only: the order and cutting of the learned schedule for given
 * per-unit costs (a unit = 16 consecutive iterations of the cell-ordered loop;
 * costs are rounded to integers >= 1).  perm_out (host, n) receives the units
 * in descending cost on a logarithmic key (32 steps per doubling; ties keep
 * unit order); starts_out (host, cap) the chunk boundaries in units of that
 * order, n_chunks + 1 entries: factoring on cost, batch b cutting P chunks of
 * ceil(R_b / (x P)) cost from the R_b left.  This is the host statement of
 * what si_generate computes on the device for SI_SCHED_LEARNED.
 */
si_status si_learned_table(const float* unit_cost, int64_t n, int32_t P, float fac_divisor,
                           int32_t* perm_out, int64_t* starts_out, int64_t cap,
                           int64_t* n_chunks);

/*
 * Host-only: from now on, on the calling thread, si_generate and
 * si_generate_batched record begin_event (a hipEvent_t) on their stream
 * immediately before the spin-image kernel launch and end_event immediately
 * after it, so a caller can time that kernel alone without synchronising.
 * NULL, NULL turns this off.  The events are owned by the caller.
 */
si_status si_set_kernel_events(void* begin_event, void* end_event);

/*
 * Host-only, for experiments on heterogeneous workers (Section 5.2 runs the
 * techniques on a mix of faster and slower processors): from now on, on the
 * calling thread, every `every`-th persistent workgroup of si_generate and
 * si_generate_batched behaves as a worker `slowdown` times slower -- after
 * each chunk it idles for (slowdown - 1) times that chunk's own time.  Work
 * and images are unchanged; the launches use a separate build of the
 * kernel.  every = 0 or slowdown = 1 turns it off.  Returns SI_E_INVALID for
 * every < 0 or a slowdown below 1 or not finite.
 */
si_status si_set_emulated_workers(int32_t every, float slowdown);

/*
 * Host-only, from now on, on the calling thread: how the emulated slower
 * workgroups of si_set_emulated_workers spend their extra time and which
 * they are.
 *   busy       0: sleeping, which leaves the compute unit to other
 *              workgroups (the default); 1: every thread spinning on
 *              arithmetic, which keeps the compute unit occupied, as a
 *              slower processor would be.  The extra time is spent after
 *              each group of images that shares a candidate pass.
 *   placement  SI_EMU_EVERY (0): workgroups k with k mod every = 0 (the
 *              default); SI_EMU_FIRST (1): the P / every workgroups whose
 *              first chunk comes first in claim order; SI_EMU_LAST (2):
 *              those whose first chunk comes last -- the order in which the
 *              paper's slower processors first requested work (Section 5.2).
 *              With FIRST or LAST, SI_SCHED_WF takes equal weights unless
 *              si_set_worker_weights gives them.
 * Returns SI_E_INVALID for other values.
 */
enum { SI_EMU_EVERY = 0, SI_EMU_FIRST = 1, SI_EMU_LAST = 2 };
si_status si_set_emulated_mode(int32_t busy, int32_t placement);

/*
 * Host-only: relative speeds of the persistent workgroups for SI_SCHED_WF,
 * from now on, on the calling thread: workgroup k takes weight
 * weights[k mod n] (host array of n positive finite values; scaled so the
 * launch's weights sum to its workgroup count).  n = 0 clears it (weights
 * then come from si_set_emulated_workers, 1 / slowdown for the slow ones, or
 * are all 1).  Returns SI_E_INVALID for n < 0, NULL with n > 0, or a weight
 * that is not positive and finite.
 */
si_status si_set_worker_weights(const float* weights, int32_t n);

/*
 * Host-only, the chunk rules of SI_SCHED_WF / AWF / AF as the kernel
 * evaluates them (the same code):
 *   si_rule_wf_chunk   ceil(w base), in [max(1, min_chunk), remaining]
 *   si_rule_awf_weight P rate / (rate_sum P / n_meas); 1 when unmeasured
 *   si_rule_af_chunk   (D + 2TR - sqrt(D^2 + 4DTR)) / (2 mu) rounded up, in
 *                      [max(1, min_chunk), R], with D and T from the sums
 *                      var_over_mu_sum, inv_mu_sum over n_meas of P workers
 */
int64_t si_rule_wf_chunk(double w, int64_t base, int64_t remaining, int32_t min_chunk);
double si_rule_awf_weight(double rate, double rate_sum, int32_t n_meas, int32_t P);
int64_t si_rule_af_chunk(double var_over_mu_sum, double inv_mu_sum, int32_t n_meas, int32_t P,
                         int64_t remaining, double mu, int32_t min_chunk);

/*
 * si_generate without allocation, for callers that cannot allocate device
 * memory: tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments and results as si_generate (images and counts identical to its
 * for the same scene, indices, params and schedule), without statistics.  What si_generate allocates per call (the
 * claim counter, the chunk table, the temporaries of the cell-sorted loop
 * order) lives in one static device array of SI_NOALLOC_SCRATCH_BYTES that
 * each device holds from the library's load until the process ends; the
 * call allocates no device or pinned memory.
 *   sched->kind  any fixed schedule; SI_SCHED_LEARNED returns
 *                SI_E_UNSUPPORTED (its plan needs memory of its own)
 * Scratch needed: 256 + 12 n_chunks bytes (each region rounded up to 256),
 * plus 4 (3N + 2M + ceil(M / 2048) + 2) bytes when the loop is cell-ordered
 * (sched->order SPREAD or CELL on a scene with more than one cell); a call
 * needing more returns SI_E_INVALID and names the size.  With 64 MiB, a
 * 2,000,000-point scene with all points oriented fits under every schedule,
 * SS with one image per chunk included (64.0e6 bytes).
 * Every call on a device reuses that device's array and leaves its contents
 * behind: calls that overlap on one device (other streams, other threads)
 * race and must not be issued.  The chunk table is computed on the host
 * into one of four vectors kept per thread and copied with hipMemcpyAsync
 * on hip_stream; a call first waits for the upload made four calls before
 * from the same vector (events created at the thread's first calls), so
 * up to four calls are queued before the host waits.  Because a graph would
 * replay that copy from storage later calls refill, a hip_stream that is
 * capturing returns SI_E_UNSUPPORTED before anything is enqueued (as for
 * si_generate).  Invalid indices are reported by si_device_errors.
 */
#define SI_NOALLOC_SCRATCH_BYTES (64u << 20)
si_status si_generate_noalloc(const si_scene* scene, const int32_t* oriented_idx, int64_t N,
                              const si_params* params, const si_sched* sched,
                              float* images_out, uint32_t* counts_out, void* hip_stream);

/*
 * The device-side error flag of the generation launches (Section 2.1's
 * loop takes P = OP[i]; an index outside the scene has no image).  Waits for
 * the work queued on hip_stream, then returns SI_E_INVALID if any generation
 * launch (si_generate, si_generate_batched, si_generate_noalloc) on the
 * current device met an oriented index outside [0, M) since the previous
 * si_device_errors call, else SI_OK.  The flag is one per device, shared by
 * all streams, and this call clears it.  Synchronises the stream.
 */
si_status si_device_errors(void* hip_stream);

const char* si_status_string(si_status status);
const char* si_last_error(void);
int32_t si_abi_version(void);

/*
 * Mesh resolution of a scene: the mean, over the chosen points, of the
 * distance from a point to its nearest other point of the scene (the paper
 * sets the bin size B as a factor of the mesh resolution, Section 2.1 and
 * the notation table; a bin of B = factor x this value).  Exact nearest
 * neighbours: each query searches the scene's grid in shells of cells until
 * no unsearched point can be nearer (a scene built with radius <= 0 is one
 * cell: brute force over M points per query).
 *   idx      device, n int32 indices of the query points (the order given
 *            to si_build_scene), or NULL for all M points (n ignored)
 *   nn_out   device, n float32 distances, or NULL
 *   mean_out host: the mean distance (FP64 sum)
 * A point at the same place as another has distance 0.  Synchronises the
 * stream.  Returns SI_E_INVALID for M < 2, n out of [1, 2^31 - 1), an
 * index outside [0, M) (its distance is NaN), or a NULL mean_out.
 */
si_status si_mesh_resolution(const si_scene* scene, const int32_t* idx, int64_t n,
                             float* nn_out, double* mean_out, void* hip_stream);

/*
 * Normals of raw points, for scenes without them (the paper's oriented
 * points come with known normals, Section 2.1): for each point p, the
 * points x with |x - p| <= radius (p included; the test |x - p|^2 <= r^2 in
 * float32), their covariance about their centroid (FP64 sums), and the unit
 * eigenvector of its smallest eigenvalue, signed so that n . (p - v) >= 0
 * for the viewpoint v (pointing away from it).  A neighbourhood whose
 * covariance is a multiple of the identity (e.g. the point alone) gets
 * (0, 0, 1) signed the same way.
 *   points_xyz   device, M x 3 float32
 *   viewpoint    host, 3 floats
 *   normals_out  device, M x 3 float32 (may not alias points_xyz)
 *   counts_out   device, M int32 neighbour counts, or NULL
 * Builds a temporary grid of cell edge >= radius on hip_stream and frees it
 * at the end, which synchronises the device.  Returns SI_E_INVALID for M
 * out of [1, 2^31 - 1), a radius that is not positive and finite, or NULL
 * or non-finite arguments.
 */
si_status si_estimate_normals(const float* points_xyz, int64_t M, float radius,
                              const float* viewpoint, float* normals_out, int32_t* counts_out,
                              void* hip_stream);

/*
 * Spin-image matching: the normalised linear correlation coefficient of
 * every pair of images from two sets (the comparison by which spin images
 * are matched in object recognition, Johnson and Hebert, cited by the paper)
 *     R(P, Q) = (N sum p q - sum p sum q)
 *               / sqrt((N sum p^2 - (sum p)^2) (N sum q^2 - (sum q)^2))
 * over all N = n_bins bins; an image with no variance has R = 0.
 *   A        device, n_a x n_bins float32 (e.g. si_generate's images_out)
 *   B        device, n_b x n_bins float32
 *   R_out    device, n_a x n_b float32 row-major, or NULL
 *   best_out device, n_a int32: for each image of A, the image of B of
 *            largest R (lowest index on ties), or NULL
 *   best_R_out device, n_a float32: that R, or NULL
 * At least one output must be given.  sum p q runs on the matrix cores in
 * fp16 with fp32 accumulation: each image is scaled by its largest |bin|
 * (R is unchanged by that) and rounded to fp16, and all sums are taken from
 * the rounded values.  Rounding moves R by at most about
 * 2u (1 + |R|) (k_P + k_Q), u = 2^-11, k = sqrt(1 + mean^2 / variance) of
 * the image's bins.  Bins must be finite.  A and B may be the same array
 * (then, with n_a = n_b, it is converted once).  Asynchronous on
 * hip_stream; the temporaries (fp16 copies, 2 n_bins bytes per image) come
 * from the device's stream-ordered pool.  n_a or n_b = 0 does nothing.  Returns
 * SI_E_INVALID for negative sizes, sizes of 2^31 - 1 or more, n_bins out of
 * [2, 65536], NULL inputs or no output.
 */
si_status si_correlate(const float* A, int64_t n_a, const float* B, int64_t n_b,
                       int32_t n_bins, float* R_out, int32_t* best_out, float* best_R_out,
                       void* hip_stream);

/*
 * Measured throughput ceilings of the device, for reading the spin kernel's
 * roofline (the VALU lane-operations of its pair tests and binning, its LDS
 * atomics, its HBM image stores).  One warm-up and one timed launch, HIP
 * events; synchronises the stream.  *value (host) receives
 *   SI_PROBE_VALU                FP32 FMA lane-operations per second (16
 *                                independent chains per lane, no packed
 *                                instructions: the code the kernel emits)
 *   SI_PROBE_LDS_ATOMIC_SEQ      ds_add_u32 per second, 64 consecutive words
 *                                per wave-instruction (conflict free)
 *   SI_PROBE_LDS_ATOMIC_RANDOM   ds_add_u32 per second, random words of a
 *                                1,024-bin image (the binning pattern)
 *   SI_PROBE_HBM_COPY            bytes per second read plus written by a
 *                                1 GiB float4 copy
 * The probe allocates and frees its own device memory (stream-ordered).
 */
enum {
    SI_PROBE_VALU = 0,
    SI_PROBE_LDS_ATOMIC_SEQ = 1,
    SI_PROBE_LDS_ATOMIC_RANDOM = 2,
    SI_PROBE_HBM_COPY = 3
};
si_status si_peak_probe(int32_t kind, double* value, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SI_H */
