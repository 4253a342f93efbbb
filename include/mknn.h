/*
 * mknn.h -- C ABI of the MI355X (gfx950) Manifold k-NN query engine.
 *
 * Method (Manifold k-NN, Sec. 3-4): points P = p_0..p_{n-1} are ordered by insertion
 * ("birth rank", 0-based: rank r is the paper's p_{r+1}).  For every rank i the successor
 * list L_i holds, ascending, the ranks j > i whose insertion pruned the Voronoi cell of p_i
 * (Sec. 3).  A k-NN query descends the lists from the oldest site to the nearest neighbour
 * (Alg. 1, collecting the "transition sites" it visits), then expands the lists of the
 * confirmed neighbours (Alg. 2, justified by Theorem 1).  Ignoring ranks >= m answers the
 * query within the prefix P_{1:m} (Sec. 4.2).  Deleting a site updates the lists locally
 * (Alg. 3, Sec. 4.3) so that they equal the lists of P minus that site inserted in the
 * original relative order.
 *
 * Results are exact with respect to squared Euclidean distances evaluated in float64 from
 * the float32 inputs as D = ((qx-px)^2 + (qy-py)^2) + (qz-pz)^2 (each operation rounded,
 * no fused multiply-add).  Neighbours are ordered by the key (D, rank): an exact tie goes to
 * the older site.  Returned distances are (float)sqrt(D).
 *
 * Conventions for every call:
 *   - the return value is an mknn_status; no C++ exception crosses this boundary;
 *     mknn_last_error() returns a thread-local message describing the last failure;
 *   - "host" pointers are ordinary CPU memory, "device" pointers are HIP device memory of
 *     the current device; the caller owns every buffer it passes in;
 *   - `stream` is a hipStream_t passed as void* (NULL = the legacy default stream); device
 *     work is enqueued on it and the call returns without synchronising unless stated.
 */
#ifndef MKNN_H_
#define MKNN_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mknn_cloud mknn_cloud; /* opaque, owned by the library */

typedef enum {
  MKNN_OK = 0,
  MKNN_EINVAL = -1,       /* bad argument (NULL pointer, size or range) */
  MKNN_ENOMEM = -2,       /* host or device allocation failed */
  MKNN_EDUPLICATE = -3,   /* two input points are bit-identical */
  MKNN_ENONFINITE = -4,   /* NaN or infinite coordinate */
  MKNN_EHIP = -5,         /* a HIP runtime call failed (message names the hipError_t) */
  MKNN_ENOTFOUND = -6,    /* deletion of an unknown or already deleted rank */
  MKNN_EBUSY = -7,        /* resource pool full; retry later */
  MKNN_EUNSUPPORTED = -8  /* valid request outside what the library supports */
} mknn_status;

/* Largest k a query may ask for. */
#define MKNN_KMAX 64

/* ---------------------------------------------------------------------------------------
 * Construction (host side).
 *
 * mknn_build: builds the successor lists of Sec. 3 by incremental Delaunay triangulation
 * (exact predicates, vertex at infinity), inserting the points in birth order.
 *   xyz    host float32 [n][3], row-major, in the caller's own order; copied.
 *   order  host int32 [n] permutation: rank r is the caller's point order[r];
 *          NULL means the identity (rank r = row r).
 *   out    receives a new cloud handle; release it with mknn_free().
 * Prefixes that span only a line or a plane are handled as the lists define them (Sec. 3):
 * cells of collinear points are slabs and cells of coplanar points prisms, so a rank joins
 * the lists of its neighbours on that line or in that plane, and the first rank off the
 * line (plane) joins the list of every older rank; a cloud may stay planar or collinear
 * throughout.  Deletion and insertion on such a cloud rebuild local triangulations that
 * need four affinely independent points and return EUNSUPPORTED where they have none.
 * Errors: EINVAL (n < 1, NULL xyz/out, order not a permutation), ENONFINITE, EDUPLICATE,
 * EUNSUPPORTED (internal construction failure), ENOMEM.
 */
mknn_status mknn_build(const float *xyz, int64_t n, const int32_t *order, mknn_cloud **out);

/* mknn_build_device: the lists of mknn_build (Sec. 3), computed on the GPU; the result is
 * the same cloud, list for list and entry for entry, as mknn_build's.  Every tetrahedron the
 * incremental construction creates is generated from pairs of tetrahedra sharing a
 * triangle, in rounds (a tetrahedron exists from its newest vertex's insertion until the
 * oldest site in its circumsphere), with the construction's own predicates: the device
 * certifies a sign with a float64 error bound and defers the rest to exact host arithmetic.
 *   xyz, order, out  as for mknn_build (host memory; copied).
 *   stream   hipStream_t as void* (NULL: the legacy default stream) for the device work;
 *            the call synchronises it and returns when the lists are on the host.
 * Device memory: about 150 bytes per point for the created tetrahedra, their ridge table
 * and the sorted entries, plus 4 bytes per conflict record (a few hundred per point);
 * freed before the call returns.  Clouds whose first four ranks are coplanar start, as in
 * mknn_build, from the first ranks off their line and plane (or spare points off them) and
 * record the lists the same way.  Clouds of fewer than five points are built by mknn_build
 * (same lists, same errors); so are those whose first two ranks coincide.
 * Errors: as mknn_build; EUNSUPPORTED for n above 2^21 - 2 (ridge keys pack three 21-bit
 * site ids); EHIP when a HIP call fails (device memory included); EDUPLICATE names the
 * first rank that repeats an older point, as mknn_build does. */
mknn_status mknn_build_device(const float *xyz, int64_t n, const int32_t *order, void *stream,
                              mknn_cloud **out);

/* Counters of the calling thread's last mknn_build_device: counts[0] rounds, [1]
 * tetrahedra created (ghosts included), [2] conflict records written, [3] candidate tests,
 * [4] tests decided exactly on the host, [5] list entries; *ms (may be NULL) the call's
 * wall time in milliseconds.  All zero when the call was handed to mknn_build.
 * Errors: EINVAL (counts NULL). */
mknn_status mknn_build_device_stats(int64_t counts[6], double *ms);

/* Number of points n of the cloud (including deleted ranks). */
int64_t mknn_size(const mknn_cloud *c);

/* Host view of the successor lists as CSR (Sec. 3, "successor table"): list i is
 * ranks[offsets[i] .. offsets[i+1]), ascending.  The pointers stay valid until the next
 * mutation of the cloud (mknn_delete) or mknn_free.  Deleted ranks have empty lists and
 * appear in no list. */
mknn_status mknn_successors(const mknn_cloud *c, const int64_t **offsets,
                            const int32_t **ranks, int64_t *nnz);

/* Host copy of the points by rank: float32 [n][3] (valid like mknn_successors). */
mknn_status mknn_points_by_rank(const mknn_cloud *c, const float **xyz);

/* ---------------------------------------------------------------------------------------
 * Device residency.
 *
 * mknn_upload: packs the lists for the device and copies them to the current device
 * (synchronously).  Layout: one 16-byte record {x, y, z, rank} per list entry, lists
 * stored contiguously in the Morton order of their owner points, and one 64-bit
 * {start, length} descriptor per rank.  Idempotent; re-uploads after a deletion.
 * Errors: EHIP, ENOMEM.
 */
mknn_status mknn_upload(mknn_cloud *c, void *stream);

/* mknn_compact: packs the device lists of an uploaded cloud again, in the upload layout,
 * which gives back the arena slack that deletion deltas have used.  Synchronises `stream`;
 * no query on the cloud may be in flight on another stream.  Errors: EINVAL (not uploaded),
 * EHIP, ENOMEM. */
mknn_status mknn_compact(mknn_cloud *c, void *stream);

/* Bytes of device memory the uploaded cloud occupies. */
int64_t mknn_device_bytes(const mknn_cloud *c);

/* ---------------------------------------------------------------------------------------
 * Queries (device side; Alg. 1 + Alg. 2 with the prefix bound of Sec. 4.2).
 *
 * mknn_knn: k nearest ranks r < m (live ranks only) of every query.
 *   d_q     device float32 [nq][3]
 *   k       1 <= k <= MKNN_KMAX;  m  1 <= m <= n (prefix size)
 *   d_idx   device int32 [nq][k]  ranks, ascending by key; -1 where fewer than k exist
 *   d_dist  device float32 [nq][k] (float)sqrt(D); +inf in padded slots
 * nq = 0 is a no-op.  The cloud must be uploaded.  Scratch for the query sort is taken from
 * the stream-ordered allocator and released on the stream.
 * Errors: EINVAL (k or m out of range, NULL pointers, not uploaded), EUNSUPPORTED
 * (k > MKNN_KMAX), EHIP.
 */
mknn_status mknn_knn(const mknn_cloud *c, const float *d_q, int64_t nq, int32_t k, int32_t m,
                     int32_t *d_idx, float *d_dist, void *stream);

/* mknn_knn_static: mknn_knn for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, rows and errors as mknn_knn, bit-identical results (the same kernels), but
 * the query sort's scratch is a fixed array of the library on each GPU
 * (256 Ki histogram bins and 256 block totals + 20 bytes per query for at most 2^20 =
 * 1,048,576 queries, about 21.0 MiB per GPU, held until the process ends) instead of
 * stream-ordered allocations:
 * the call makes no hipMalloc/hipFree and no allocating library call.  The array's device
 * address is looked up on the first call on each device.  Every call on one GPU shares that
 * GPU's array: calls whose work overlaps on one GPU (other streams, other threads) race on
 * it and must be serialised by the caller; each call clears what must start at zero.
 * Errors: as mknn_knn, and EINVAL for nq above 2^20.
 */
mknn_status mknn_knn_static(const mknn_cloud *c, const float *d_q, int64_t nq, int32_t k,
                            int32_t m, int32_t *d_idx, float *d_dist, void *stream);

/* mknn_knn_layout: mknn_knn with k = 16 and m = n over another layout of the same lists,
 * for callers that measure the device layout (Sec. 3's successor table is kept as 16-byte
 * records {x, y, z, rank} that inline each entry's coordinates):
 *   MKNN_LAYOUT_RANKS   a 4-byte rank per entry, the point then gathered by rank;
 *   MKNN_LAYOUT_ARRAYS  four arrays of 4-byte values per entry: rank, x, y, z.
 * Same rows as mknn_knn, bit for bit; the query kernel is timed by mknn_timing_* like
 * mknn_knn's.  The arrays (4 or 16 bytes per record) are built from the records and freed
 * on `stream` in the call.
 * Errors: as mknn_knn; EINVAL for another layout; EUNSUPPORTED while deletions are pending
 * (mknn_delete_lazy). */
#define MKNN_LAYOUT_RANKS 1
#define MKNN_LAYOUT_ARRAYS 2
mknn_status mknn_knn_layout(const mknn_cloud *c, int32_t layout, const float *d_q, int64_t nq,
                            int32_t *d_idx, float *d_dist, void *stream);

/* mknn_knn_var: per-query k and prefix m with ragged output rows.
 *   d_k        device int32 [nq], each in [1, MKNN_KMAX]
 *   d_m        device int32 [nq], each in [1, n] (values above n are clamped to n)
 *   d_row_off  device int64 [nq+1]; row q occupies [d_row_off[q], d_row_off[q+1]) of
 *              d_idx / d_dist, and d_row_off[q+1] - d_row_off[q] must equal d_k[q]
 *   kmax       host int32, an upper bound of all d_k (selects the kernel variant)
 * Before the query runs, a small kernel checks every query's k, m and row length on the
 * device and the call reads the verdict back, so it synchronises `stream` once.
 * Errors as mknn_knn, and EINVAL (nothing written) if some query has k outside [1, kmax],
 * m < 1, or d_row_off[q+1] - d_row_off[q] != d_k[q]; the message names the first such
 * query.
 */
mknn_status mknn_knn_var(const mknn_cloud *c, const float *d_q, int64_t nq, const int32_t *d_k,
                         const int32_t *d_m, const int64_t *d_row_off, int32_t kmax,
                         int32_t *d_idx, float *d_dist, void *stream);

/* ---------------------------------------------------------------------------------------
 * Batched form: many clouds with their own query sets, k and prefixes in one launch per
 * register class (k <= 16, 32, 48, 64).  Same per-query semantics as mknn_knn (Alg. 1 +
 * Alg. 2, Sec. 4.2).
 *
 * The queries of all requests are bucketed together by (request, Morton code) unless
 * MKNN_BATCH_NO_SORT is set.  By default each class is one flat launch over its requests
 * laid end to end: every wavefront takes four consecutive sorted queries of one request,
 * the workgroups of a batch spread evenly and contiguously over the 8 XCDs.  With the
 * environment variable MKNN_BATCH_PERSISTENT=1 at plan creation, that plan uses a
 * persistent launch instead: each
 * request is cut into tiles of at most `tile_queries` queries (4 .. 2^20; 16 is a good
 * default), requests go to 8 per-XCD queues (largest estimated cost first), and persistent
 * wavefronts claim tiles from their own queue with an atomic counter and steal from the
 * others when it runs dry.  `tile_queries` only matters for the persistent launch.
 */
typedef struct {
  const mknn_cloud *cloud;   /* an uploaded cloud */
  const float *d_q;          /* device float32 [nq][3] */
  int64_t nq;                /* >= 0 */
  int32_t k;                 /* 1..MKNN_KMAX */
  int32_t m;                 /* prefix size in [1, n]; 0 means n */
  int32_t *d_idx;            /* device int32 [nq][k], rows as in mknn_knn */
  float *d_dist;             /* device float32 [nq][k] */
} mknn_request;

typedef struct mknn_batch_plan mknn_batch_plan; /* opaque, owned by the library */

#define MKNN_BATCH_NO_SORT 1   /* skip the Morton bucketing of the queries */
#define MKNN_BATCH_NO_GRAPH 2  /* launch eagerly instead of replaying a captured hipGraph */

/* mknn_batch_plan_create: device buffers for up to max_requests requests and max_queries
 * queries in total (max_queries < 2^31), plus pinned host staging.  Unless
 * MKNN_BATCH_NO_GRAPH is set, the first run captures the whole sequence (descriptor copy,
 * counter clear, query bucketing, the launches of the register classes that have work)
 * into a hipGraph.  Later runs update the descriptors in the pinned staging area and replay
 * the graph: every kernel reads its sizes from device memory and uses a fixed grid; a run
 * with work in a class the graph does not launch captures the graph again, with that class
 * added.  A plan belongs to the device that was current at creation.
 * Errors: EINVAL, ENOMEM, EHIP. */
mknn_status mknn_batch_plan_create(int64_t max_requests, int64_t max_queries,
                                   int32_t tile_queries, int32_t flags, mknn_batch_plan **out);

/* mknn_batch_plan_run: enqueue one batch on `stream`.  The request array (host) is read
 * before returning.  Outputs are written asynchronously.  A run waits for the previous
 * run of the same plan to finish using the staging area.  Errors: EINVAL (bad request or
 * over capacity), EUNSUPPORTED (k > MKNN_KMAX), EHIP.  Requests with nq = 0 are skipped. */
mknn_status mknn_batch_plan_run(mknn_batch_plan *plan, const mknn_request *reqs, int32_t nreq,
                                void *stream);

/* Autotuner of the plan's own launch, on this batch (three timed runs per candidate after a
 * warm-up, HIP events on `stream`).  Flat launch (the default): the merge threshold of
 * every register class with work (candidates per chunk from which the merge network
 * replaces one-by-one insertion: 4, 6, 8 for k <= 16; 5, 8, 11, 14, 17 above), one class
 * at a time; the plan keeps the fastest per class, and *best receives the threshold of the
 * class with the most queries.  Persistent launch: the tile length (8, 16, 32, 64, 256);
 * the plan keeps the fastest and *best receives it.  The outputs hold the batch's results
 * afterwards. */
mknn_status mknn_batch_plan_tune(mknn_batch_plan *plan, const mknn_request *reqs, int32_t nreq,
                                 void *stream, int32_t *best);

/* Release a plan (waits for its last run). */
void mknn_batch_plan_destroy(mknn_batch_plan *plan);

/* Convenience form: runs the batch on a plan the library keeps per process and grows on
 * demand.  Not thread-safe. */
mknn_status mknn_batch_knn(const mknn_request *reqs, int32_t nreq, void *stream);

/* ---------------------------------------------------------------------------------------
 * Autotuner.
 *
 * The query kernels come in three families -- one query per lane (register list of k
 * entries), 16 lanes per query in lockstep, and 16 lanes per query with every row scheduled
 * independently -- and, for k <= 16, switch from one-by-one candidate insertion to a
 * merge network above a number of candidates per chunk.  mknn_autotune times every
 * candidate configuration on the given queries (device float32 [nq][3], k, prefix m; m = 0
 * means n) with HIP events on `stream`, keeps the fastest for clouds of this size class
 * (log2 n) and this k class on the current device, and reports the timings.  Later
 * mknn_knn / mknn_knn_var launches and batch plans use the table; untuned classes use the
 * built-in defaults.  The table lives in the process and can be saved and loaded as text.
 *   tried      optional host array of max_tried entries, receives every candidate
 *   ntried     number of candidates timed
 *   best       the chosen configuration
 * Errors: EINVAL, EUNSUPPORTED (k), EHIP.  Not thread-safe with concurrent launches on the
 * same stream.
 */
typedef struct {
  int32_t family;      /* 1 lane per query, 2 lockstep rows, 3 scheduled rows */
  int32_t merge_min;   /* k <= 16: candidates per chunk from which the merge network is used */
  int32_t per_wave;    /* scheduled rows: queries per wavefront */
  float ms;            /* best of three timed runs (milliseconds) */
} mknn_tune_entry;

mknn_status mknn_autotune(const mknn_cloud *c, const float *d_q, int64_t nq, int32_t k, int32_t m,
                          void *stream, mknn_tune_entry *tried, int32_t max_tried,
                          int32_t *ntried, mknn_tune_entry *best);
/* Text form of the table: a "mknn-tune 1" line, then one line per entry
 * "device S exact log2n family merge_min per_wave".  Load merges into the current table.
 * Errors: EINVAL (path, malformed file), ENOTFOUND (load: no such file). */
mknn_status mknn_tune_save(const char *path);
mknn_status mknn_tune_load(const char *path);
void mknn_tune_reset(void);

/* ---------------------------------------------------------------------------------------
 * k-NN with a local plane fit (the neighbourhood statistic of the paper's scan convergence
 * study, Sec. 5.3.1: a plane fitted by PCA to each probe's k nearest neighbours in a prefix).
 *
 * mknn_knn_plane: the rows of mknn_knn, and per query 8 floats in d_plane (device float32
 * [nq][8], caller-owned): the centroid c of the k' <= k neighbours found (3), the unit
 * normal (3): the eigenvector of the smallest eigenvalue l0 of their covariance
 * (1/k') sum (p - c)(p - c)^T, with its largest-magnitude component positive, the residual
 * sqrt(l0) (RMS distance of the neighbours to the plane), and the surface variation
 * l0 / (l0 + l1 + l2).  With fewer than three neighbours the last five are NaN (all eight
 * with none).  Computed in float64 (cyclic Jacobi on the 3x3 covariance) by a second kernel
 * that reads the rows just written, on the same stream.  Errors as mknn_knn.
 */
mknn_status mknn_knn_plane(const mknn_cloud *c, const float *d_q, int64_t nq, int32_t k,
                           int32_t m, int32_t *d_idx, float *d_dist, float *d_plane,
                           void *stream);

/* ---------------------------------------------------------------------------------------
 * Work counters (diagnostics for the memory roofline).
 *
 * mknn_knn_counts: runs the same query path as mknn_knn and writes, per query, the number of
 * list entries examined E and of lists opened L (int32 [nq] each, device), counted as the
 * sequential Alg. 1 + Alg. 2 would: descent scans stop at the jump entry, and the final
 * list of the descent, which Alg. 2's first iteration would scan again, is counted once.
 * d_inserts (optional, may be NULL): candidates actually inserted into N per query.
 */
mknn_status mknn_knn_counts(const mknn_cloud *c, const float *d_q, int64_t nq, int32_t k,
                            int32_t m, int32_t *d_entries, int32_t *d_lists,
                            int32_t *d_inserts, void *stream);

/* ---------------------------------------------------------------------------------------
 * Kernel timing (diagnostics for the memory roofline).
 *
 * mknn_timing_enable(1): from now on every query call records a pair of HIP events on its
 * stream immediately before and after its main query kernel (the query sort is outside the
 * pair).  mknn_timing_read() waits for all recorded pairs, returns the summed kernel time in
 * milliseconds and the number of launches, and forgets them.  Not thread-safe: meant for
 * single-threaded benchmarking.  Errors: EHIP.
 */
mknn_status mknn_timing_enable(int enable);
mknn_status mknn_timing_read(double *total_ms, int64_t *launches);

/* ---------------------------------------------------------------------------------------
 * Memory probes (diagnostics for the memory roofline of the query kernels; the paper has no
 * counterpart).
 *
 * mknn_probe_stream_read: sustained rate of a streaming read of the caller's device buffer
 * (`bytes`, a multiple of 16, at least 4 KiB; make it larger than the 256 MB last-level
 * cache to measure HBM).  mknn_probe_gather16: sustained rate of `accesses` (rounded up to
 * a multiple of 16,384) random 16-byte record reads from the buffer (its largest
 * power-of-two number of records), counting 16 useful bytes per read -- the access of a
 * list walk that opens a new list.  Both run one untimed and `reps` timed launches on
 * `stream` (HIP events; synchronises) and report the best in *gbps (1e9 bytes per second).
 * The buffer is only read.  Errors: EINVAL, EHIP.
 */
mknn_status mknn_probe_stream_read(const void *d_buf, int64_t bytes, int32_t reps, void *stream,
                                   double *gbps);
mknn_status mknn_probe_gather16(const void *d_buf, int64_t bytes, int64_t accesses, int32_t reps,
                                void *stream, double *gbps);

/* ---------------------------------------------------------------------------------------
 * Deletion (Sec. 4.3, Alg. 3).
 *
 * mknn_delete: removes the given live ranks, one after the other.  Afterwards the successor
 * lists equal those of the remaining points inserted in the original relative order.
 * Method: prune the deleted rank from its predecessors' lists (Lemma 1).  Then, for every
 * entry k of its list, rebuild the local Delaunay triangulation of its former neighbours
 * and add each pair (j, k) whose shared Voronoi facet reaches into the deleted site's old
 * cell (Lemma 2).  Ranks keep their numbers; deleted ranks disappear from all lists, and
 * the head moves to the oldest live rank.  m keeps counting original ranks.
 * If the cloud is uploaded, the changed lists are copied on write into fresh segments of
 * the device arena and their descriptors are switched by a kernel on `stream`.  Work
 * enqueued later on that stream sees the new lists; work already running keeps reading
 * the old segments.  When the arena's slack runs out, the lists are packed again.  The
 * call synchronises `stream` before returning.
 *   ranks  host int32 [count]
 * The batch is reordered into rounds of deletions whose local sets (the rank, its
 * predecessors and its list) are pairwise disjoint -- they commute, since the result is
 * defined by the remaining points alone -- and the host work of a round runs on several
 * threads (at most OMP_NUM_THREADS, else the hardware threads, shared by every call in the
 * process); the lists are those of the serial order.
 * Errors: ENOTFOUND (unknown, deleted or repeated rank; nothing is changed), EINVAL (the
 * last live point), EUNSUPPORTED (the local set starts with four coplanar points; the ranks
 * applied before the failing one -- earlier rounds, and earlier ranks of its round in batch
 * order -- stay deleted on the host, and the device copy must be uploaded again before the
 * next query), EHIP, ENOMEM.  Not thread-safe per cloud: queries on other streams must be
 * ordered around a deletion by the caller.
 */
mknn_status mknn_delete(mknn_cloud *c, const int32_t *ranks, int64_t count, void *stream);

/* mknn_delete_lazy: marks live ranks as deleted without running Alg. 3 yet.  The marks are a
 * device bitmap (one bit per rank, allocated on the first call and grown by re-allocation)
 * set by a kernel on `stream`; the call synchronises `stream`.  Until they are applied,
 * every query on the cloud (mknn_knn, mknn_knn_plane, mknn_knn_var, mknn_batch_plan_run)
 * walks the un-updated lists for min(MKNN_KMAX, k + 16) neighbours and keeps the first k
 * unmarked ones.  These are the k nearest remaining ranks whenever the walk found at least
 * k unmarked ones (every site outside the walk's list is farther than all of it); a row with
 * fewer is exact only if the prefix holds fewer sites than the walk's width.  Otherwise the
 * call applies the pending deletions (as mknn_delete: host Alg. 3, then the delta; it
 * synchronises `stream`) and answers again, so every result is exact.  A query call with
 * marks pending reads one word back from the device and therefore synchronises `stream`.
 * mknn_delete applies the pending marks together with its own batch; mknn_insert,
 * mknn_knn_counts, mknn_autotune and a re-upload apply them first; mknn_knn_static returns
 * EUNSUPPORTED while marks are pending (it must not allocate, and applying them does).
 * mknn_live_count no longer counts marked ranks.
 *   ranks  host int32 [count]
 * Errors: ENOTFOUND (unknown, deleted, already marked or repeated rank; nothing is marked),
 * EINVAL (not uploaded; the last live point), EHIP, ENOMEM.  Not thread-safe per cloud. */
mknn_status mknn_delete_lazy(mknn_cloud *c, const int32_t *ranks, int64_t count, void *stream);

/* Applies the pending marks (Alg. 3 on the host, then the delta on `stream`, which is
 * synchronised).  Errors as mknn_delete; if Alg. 3 fails part way (EUNSUPPORTED) the
 * pending set is dropped: the ranks applied before the failing one stay deleted, the rest
 * stay live, and the cloud must be uploaded again.  No pending marks: a no-op. */
mknn_status mknn_delete_flush(mknn_cloud *c, void *stream);

/* Number of ranks marked by mknn_delete_lazy and not yet applied. */
int64_t mknn_pending_deletes(const mknn_cloud *c);

/* ---------------------------------------------------------------------------------------
 * Insertion (the construction of Sec. 3, continued).
 *
 * mknn_insert: appends `count` points (host float32 [count][3]) to the birth order as ranks
 * n, n+1, ...; their caller ids are their ranks.  Afterwards the successor lists equal those
 * of the live points plus the new ones inserted in rank order: each new rank is appended to
 * the lists of its Delaunay neighbours among the live points (and earlier new points), and
 * its own list starts empty.  The triangulation of the live points is built at the first
 * insertion and kept in the cloud (a few hundred bytes per point); deletions remove their
 * points from it (if one cannot, it is dropped and the next insertion builds it again).
 * If the cloud is uploaded, the changed lists and the new descriptors are applied on
 * `stream` as for deletions (copy on write; a re-pack when the slack runs out); the call
 * synchronises `stream` before returning.
 *   xyz    host float32 [count][3]; copied.
 * Errors: ENONFINITE, EDUPLICATE (a point coincides with a live point or another new
 * point; nothing is changed in either case), EUNSUPPORTED (fewer than four live points or
 * more than 2^30 points: nothing is changed; or a failed insertion: the points before it
 * stay inserted on the host, and the device copy must be uploaded again before the next
 * query), EHIP, ENOMEM.  Not thread-safe per cloud, like mknn_delete.
 */
mknn_status mknn_insert(mknn_cloud *c, const float *xyz, int64_t count, void *stream);

/* Number of live points, and the oldest live rank (where every descent starts). */
int64_t mknn_live_count(const mknn_cloud *c);
int32_t mknn_head(const mknn_cloud *c);

/* ---------------------------------------------------------------------------------------
 * Serving: continuous batching over resident clouds, deletions (and insertions) between
 * batches.
 *
 * A server owns `nstreams` stream slots (default priority) and a scheduler thread.
 * Requests and deletion batches are queued in arrival order.  Whenever a slot is free, the
 * scheduler forms a wave from the waiting requests, in order, while the wave's queries fit
 * the slot's share of `pool_queries` (admission by memory footprint) and it holds at most
 * `max_wave_requests` requests.  The wave runs as one batched launch on that slot.  Waves
 * on different slots overlap on the GPU, and requests arriving meanwhile join the next
 * wave.  Deletion batches on one cloud run one at a time in arrival order: the host part
 * (Alg. 3) on a worker thread while waves continue, then the device delta, ordered after
 * the in-flight waves that read the cloud.  By default a request answers on exactly the
 * deletions submitted before it (a deletion waits for earlier requests on its cloud to be
 * launched, and later requests on that cloud wait for the deletion).  With
 * MKNN_SERVER_BIND_AT_ADMISSION a request answers on the lists current when its wave is
 * launched, and never waits for a deletion's host part.
 * MKNN_SERVER_LAZY_DELETE keeps that strict order without making requests wait for the
 * host part of a deletion.  A deletion batch takes the next epoch of its cloud and is
 * checked (as mknn_delete checks it; a bad batch fails whole) and marked in the cloud's
 * device epoch array at once, on a marking stream, after any insertion queued before it
 * has been applied.  A request over-fetches and filters the marks of the epochs submitted
 * before it (mknn_delete_lazy describes the filter), so later deletions never touch its
 * answer.  An update's device delta is applied only once every request submitted before
 * it has completed, and a request with a row the filter could not certify is queued again
 * and answered once the deletions it saw are applied.  Insertions are handled as in the
 * strict order.  Not with MKNN_SERVER_PLAIN or MKNN_SERVER_BIND_AT_ADMISSION (EINVAL), and
 * not on a cloud with deletions pending from mknn_delete_lazy (EINVAL at submission).
 * With MKNN_SERVER_PLAIN (the per-request baseline) every request is its own mknn_knn
 * launch, back to back in arrival order on one stream, at most 64 in flight and together
 * at most pool_queries queries; nstreams and max_wave_requests are then ignored.
 * Request buffers are caller-owned and must stay valid until the request completes.  If
 * h_idx/h_dist (pinned host memory, [nq][k]) are given, the results are copied there before
 * the request counts as complete.
 */
typedef struct mknn_server mknn_server;

#define MKNN_SERVER_PLAIN 1
#define MKNN_SERVER_BIND_AT_ADMISSION 2
#define MKNN_SERVER_LAZY_DELETE 4

mknn_status mknn_server_create(int64_t pool_queries, int32_t nstreams, int32_t max_wave_requests,
                               int32_t flags, mknn_server **out);
/* Queue a request; *ticket identifies it.  Errors: EINVAL, EUNSUPPORTED (k), EBUSY (a single
 * request larger than a slot's pool). */
mknn_status mknn_server_submit(mknn_server *s, const mknn_request *req, int32_t *h_idx,
                               float *h_dist, uint64_t *ticket);
/* Queue a deletion batch (host int32 ranks, copied). */
mknn_status mknn_server_delete(mknn_server *s, mknn_cloud *c, const int32_t *ranks, int64_t count,
                               uint64_t *ticket);
/* Queue an insertion batch (host float32 [count][3], copied; see mknn_insert).  Insertion
 * and deletion batches of one cloud are one ordered stream of update batches, handled
 * exactly like the deletions above; the new points take the ranks from the cloud's size
 * when the batch is applied, so batches on one cloud number their points in arrival
 * order. */
mknn_status mknn_server_insert(mknn_server *s, mknn_cloud *c, const float *xyz, int64_t count,
                               uint64_t *ticket);
/* *done = 1 once the operation has completed. */
mknn_status mknn_server_poll(mknn_server *s, uint64_t ticket, int32_t *done);
/* Block until the operation completes, then forget the ticket.  times (may be NULL)
 * receives, in seconds of mknn_server_now(): [0] submission, [1] launch (a request's wave
 * was launched; a deletion's device delta was enqueued), [2] completion observed (after the
 * copies to host memory).  updates_seen (may be NULL) receives, for a request, the number
 * of update batches (deletions and insertions) of this server applied to its cloud when it
 * was launched (with MKNN_SERVER_LAZY_DELETE: submitted on its cloud before it and not
 * failed -- the ones its answer reflects).  Returns the operation's own status. */
mknn_status mknn_server_wait(mknn_server *s, uint64_t ticket, double *times,
                             int64_t *updates_seen);
/* Waves launched so far and the requests they held. */
mknn_status mknn_server_stats(mknn_server *s, int64_t *waves, int64_t *wave_requests);
/* Monotonic clock of the server, in seconds. */
double mknn_server_now(void);
/* Finish every queued operation, then release the server. */
void mknn_server_destroy(mknn_server *s);

/* Release a cloud and all its host and device memory (device frees synchronise). */
void mknn_free(mknn_cloud *c);

/* Thread-local description of the last error ("" if none). */
const char *mknn_last_error(void);

/* Library version string. */
const char *mknn_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MKNN_H_ */
