/*
 * lider.h -- C ABI of the MI355X (gfx950) LIDER library.
 *
 * LIDER (arXiv 2205.00970) is a two-layer learned index for dense retrieval:
 * k-means clusters the corpus (Section 3.2); a "centroids retriever" core model
 * indexes the centroids and one "in-cluster retriever" core model indexes each
 * cluster (Section 3.3.2).  A core model hashes vectors with SK-LSH, sorts the
 * hash keys, re-scales them (Section 5.1, Eq. (8)) and trains a two-stage linear
 * RMI (Section 5.2) that predicts a key's location in the sorted array; a search
 * scans a fixed-length window around the predicted location and scores the
 * candidates exactly (Section 3.3.1).
 *
 * Conventions for every entry point:
 *  - Pointers named *_dev are device pointers (hipMalloc'd, e.g. a torch CUDA
 *    tensor's data_ptr) on the current HIP device; *_host are host pointers.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - Matrices are dense row-major; a "row" is one d-dimensional fp32 vector.
 *  - Return value: LIDER_OK (0) or a negative lider_status.  On error a
 *    description is available from lider_last_error() on the same thread.
 *    Arguments are validated before anything is enqueued; an invalid call
 *    enqueues nothing.  Faults of already-enqueued device work surface as
 *    LIDER_EDEVICE from a later call or from the caller's stream sync.
 *  - No C++ exception crosses this boundary.
 */
#ifndef LIDER_H
#define LIDER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LIDER_OK = 0,
  LIDER_EINVAL = -1,  /* bad argument (null pointer, size out of range, ...) */
  LIDER_ENOMEM = -2,  /* device allocation failed (build only) */
  LIDER_EDEVICE = -3, /* a HIP runtime call failed */
  LIDER_ERANGE = -4,  /* a hash value does not fit in int32 */
  LIDER_EBUSY = -5,   /* reserved */
  LIDER_EIO = -6      /* file open / read / write failed, or not an index file */
} lider_status;

typedef enum {
  LIDER_F32 = 0,     /* IEEE fp32 */
  LIDER_BF16 = 1,    /* bfloat16 (round to nearest even) */
  LIDER_FP8E4M3 = 2  /* OCP fp8 e4m3 with one fp32 scale per row */
} lider_dtype;

/* Largest supported hash count per array, hashkey arrays per core model,
 * k, and c. */
#define LIDER_MAX_M 16
#define LIDER_MAX_H 16
#define LIDER_MAX_K 1024
#define LIDER_MAX_C 128

/* Hash families (lider_build_params.hash_kind). */
#define LIDER_HASH_E2LSH 0
#define LIDER_HASH_SIGN 1

typedef struct lider_index lider_index; /* opaque; owns its device memory */

/* Build parameters (Sections 3.2, 3.3, 5).
 *  n_clusters     number of k-means clusters c of Table 1 (1..n).
 *  m              hashes per key M of Table 1 (1..LIDER_MAX_M), per array.
 *  n_arrays       hashkey arrays H per core model (Section 3.3.1; 0 means 1,
 *                 at most LIDER_MAX_H).  Each array has its own hash functions,
 *                 sorted array and RMI; a search scans one window per array and
 *                 scores the union of the windows (each item once).  With H > 1
 *                 no cluster may hold more than 65536 rows.
 *  w              E2LSH bucket width (> 0): digit = floor((a.x + b) / w).
 *  rmi_fanout     second-stage width W_i of the in-cluster RMIs (Section 7.2.1).
 *  rmi_fanout_l1  second-stage width W_c of the centroids retriever (0 = same).
 *  lsh_a_host     [2Hm x d] fp32 projections: rows h*m..h*m+m-1 hash array h
 *                 of the centroids retriever, rows H*m + h*m.. array h of
 *                 every in-cluster retriever (one set per array, shared by the
 *                 clusters).  For H = 1: rows 0..m-1 layer 1, m..2m-1 layer 2.
 *                 Copied; may be freed after the call.  NULL: drawn from
 *                 `seed` (see lider_draw_params), together with lsh_b_host.
 *  lsh_b_host     [2Hm] fp32 offsets in [0, w), same row order (required
 *                 with lsh_a_host for E2LSH).
 *  assignment_dev optional [n] int32 cluster of each row (0..n_clusters-1);
 *                 NULL runs k-means.  Empty clusters are allowed (their
 *                 centroid is the zero vector).
 *  kmeans_init_host [n_clusters] int64 row ids of the initial centroids
 *                 (distinct not required); with kmeans_seeding = 1 only
 *                 element 0 is read.  NULL (and assignment_dev NULL): drawn
 *                 from `seed` (see lider_draw_params).
 *  kmeans_iters   maximum Lloyd iterations (>= 1); stops early when an
 *                 assignment repeats the previous one.
 *  storage        LIDER_F32, or LIDER_BF16 to add a bf16 copy of the corpus
 *                 for the precision form (the fp32 copy is always kept).
 *  centroid_storage LIDER_F32, or LIDER_FP8E4M3 to add per-row-scaled fp8
 *                 centroids for precision-form routing.
 *  kmeans_seeding 0: initial centroids are the rows kmeans_init_host[0..C).
 *                 1: farthest-first traversal -- the first centroid is row
 *                 kmeans_init_host[0], each next one the row farthest (squared
 *                 Euclidean, decided in FP64, ties to the smaller id) from its
 *                 nearest chosen centroid.
 *  hash_kind      LIDER_HASH_E2LSH: integer digits floor((a.x + b) / w), keys
 *                 mixed-radix over each model's digit box.  LIDER_HASH_SIGN:
 *                 the cosine variant of Section 4.1 -- one bit per hash,
 *                 1 if a.x >= 0 else 0 (decided in FP64 like the digits; w and
 *                 lsh_b_host are ignored, lsh_b_host may be NULL), key =
 *                 Decimal(bits) (Section 5.1), i.e. the box is [0, 1] for
 *                 every bit.  Use on normalised embeddings (inner product =
 *                 cosine similarity).
 *  seed           seed of the draws the caller leaves to the library (the
 *                 hash parameters when lsh_a_host is NULL, the k-means seed
 *                 rows when kmeans_init_host is NULL); ignored otherwise. */
typedef struct {
  int32_t n_clusters;
  int32_t m;
  int32_t rmi_fanout;
  int32_t rmi_fanout_l1;
  double w;
  const float* lsh_a_host;
  const float* lsh_b_host;
  const int32_t* assignment_dev;
  const int64_t* kmeans_init_host;
  int32_t kmeans_iters;
  int32_t storage;
  int32_t centroid_storage;
  int32_t kmeans_seeding;
  int32_t hash_kind;
  int32_t n_arrays;
  uint64_t seed;
} lider_build_params;

/* Build an index over corpus_dev [n x d] fp32 (Sections 3.2, 3.3.1, 3.3.2):
 * k-means (unless an assignment is given), layer-2 digits of every row,
 * per-cluster digit boxes and mixed-radix keys, a stable sort by
 * (cluster, key, id), key re-scaling, RMI training, and a copy of the corpus
 * reordered by that sort; then the same core model over the centroids.
 * Runs on `stream` and synchronises it before returning.  The index keeps its
 * own copy of everything; the caller may free corpus_dev afterwards.
 * n in 1..2^31-1, d in 1..65536.  Errors: EINVAL, ENOMEM, EDEVICE, ERANGE. */
int lider_build(const float* corpus_dev, int64_t n, int32_t d, const lider_build_params* params,
                void* stream, lider_index** out);

/* The library's seeded draws (host only; no device work, no allocation on the
 * device).  The random inputs of a build -- the E2LSH projections
 * a_i ~ N(0, I_d) and offsets b_i ~ U[0, w) of Section 4, and the rows that
 * seed k-means (Section 3.2) -- as lider_build draws them from `seed` when the
 * caller gives none:
 *  - words: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014); stream s (0: hash
 *    parameters, 1: k-means rows) starts from the state seed xor the (s+1)-th
 *    output of the generator started at state 0; a uniform is
 *    (word >> 11) * 2^-53.
 *  - lsh_a_host [2Hm x d] (H = n_arrays, 0 means 1), filled row by row with
 *    Box-Muller normals: each pair of uniforms (u1, u2) gives
 *    sqrt(-2 ln(1 - u1)) * cos(2 pi u2), then the same times sin(2 pi u2),
 *    computed in FP64 and rounded to fp32 (an odd count drops the last sine);
 *    then lsh_b_host [2Hm] = fp32(u * w), one uniform per row in order
 *    (LIDER_HASH_SIGN: all zero, no draws).  Both NULL: not drawn; one NULL:
 *    EINVAL.
 *  - rows_host [n_rows]: the first n_rows ids of a Fisher-Yates shuffle of
 *    0..n-1 on stream 1 (position i takes the id at i + floor(x (n - i) /
 *    2^64) for the next word x).  lider_build uses n_rows = n_clusters (1 with
 *    farthest-first seeding).  NULL: not drawn.
 * Errors: EINVAL for sizes out of range (m 1..16, d 1..65536, n_arrays 0..16,
 * w > 0 for E2LSH, 1 <= n <= 2^31-1, 0 <= n_rows <= n). */
int lider_draw_params(uint64_t seed, int32_t n_arrays, int32_t m, int32_t d, double w,
                      int32_t hash_kind, float* lsh_a_host, float* lsh_b_host, int64_t n,
                      int32_t n_rows, int64_t* rows_host);

/* Release the index and all its device memory.  NULL is a no-op.  Must not be
 * called while a search on the index is still running. */
void lider_free(lider_index* index);

/* Thread-local description of the last error (empty string if none). */
const char* lider_last_error(void);

/* Search options (lider_search_ex).  Zero-initialise for defaults.
 *  r1             layer-1 window length (0 = r): centroids scanned around the
 *                 centroids retriever's predicted location.
 *  precision      LIDER_F32: exact fp32 rerank of every window row.
 *                 LIDER_BF16: precision form -- bf16 first pass over the
 *                 windows (needs storage = LIDER_BF16), a shortlist per query,
 *                 fp32 rerank of the shortlist from the fp32 copy.  Routing is
 *                 exact as in LIDER_F32; with l1_dense = -1 on an index with
 *                 fp8 centroids the window kernel scores the fp8 copy, and the
 *                 routed set is decided from those scores with the fp8 error
 *                 bound (FP64 rescoring inside it), like the bf16 scores.
 *  shortlist_mult 0: certified shortlist -- every candidate whose bf16 score
 *                 is at least the k-th best bf16 score minus twice the bf16
 *                 error bound of the query (|q - bf16(q)| max|x| +
 *                 |bf16(q)| max|x - bf16(x)| + 2 d 2^-24 |bf16(q)| max|bf16(x)|,
 *                 the maxima over the index's rows): it contains the exact
 *                 top k, so the result is the fp32 top k of all candidates;
 *                 its length adapts per query (up to all candidates).
 *                 m > 0: the m*k best bf16 scores (m*k <= 4096; approximate).
 *  persistent     0: one wave per row tile of the whole index (tiles no window
 *                 touches exit at once).  1: a persistent grid whose waves pull
 *                 the index's tiles from per-XCD counters.  2: the tiles some
 *                 window overlaps are first collected into a work list on the
 *                 device and a persistent grid pulls only those (for small or
 *                 sparse batches on large indexes).  Results are identical.
 *  tile_rows      rows per rerank tile: 32 or 64 (one wave per tile), 128 (with
 *                 the operand-ordered copy of the precision asked for and
 *                 persistent = 0: a workgroup of 4 waves per tile, 32 rows
 *                 each, sharing the tile's pair list and each pass's query
 *                 rows through LDS; else one wave per tile), or 0: 128 when
 *                 the workgroup form applies, else 64 or 32 from the expected
 *                 number of pairs overlapping a tile.  pass_pairs 0 then
 *                 follows the same estimate.  Results are identical.
 *  l1_dense       How the layer-1 scores are computed; the routed set is then
 *                 decided exactly (the FP64 definition): the centroids whose
 *                 score lies within twice its rigorous error bound of the c-th
 *                 best window score are candidates, and unless they are
 *                 exactly c they are rescored by sequential FP64 inner
 *                 products.  0 (default): one dense query x centroid product
 *                 on MFMA in bf16 (every centroid scored; each query's window
 *                 read from its row), split when c > 1 (as 3).  1: the dense
 *                 product in fp32.  2: the plain bf16 product (bf16 roundings
 *                 of both operands).  3: the split bf16 product: each fp32
 *                 value x becomes h = bf16(x) and l = bf16(x - h), and the
 *                 score sums h_q h_mu + h_q l_mu + l_q h_mu (error about
 *                 3 2^-16 |q| |mu| instead of 2^-7 |q| |mu|: far fewer
 *                 candidates to rescore when c > 1; needs d a multiple of 64
 *                 and 16-byte aligned queries, else acts as 2).  -1: the
 *                 window kernel (fp32 scores of the r1-windows only).  The
 *                 routed sets, and so all results, are identical.  With
 *                 n_arrays > 1, -1 acts as 1; with r1 < n_clusters the routing
 *                 runs over the union of the H windows (at most 65536
 *                 clusters).  The dense product needs nq x n_clusters floats
 *                 of workspace.
 *  grid_mult      persistent grid: grid_mult waves per SIMD, i.e. 4 * grid_mult *
 *                 number of CUs one-wave workgroups (0 = 4).
 *  expand_bits    0: fixed window of r (r1) positions, floor(r/2) left of the
 *                 predicted location (shifted inward at the ends).  B in 1..16:
 *                 dist_e-guided expansion (Section 4.2, C = 2^B), only for
 *                 LIDER_HASH_SIGN indexes -- from the predicted location the
 *                 range grows on the side whose next hashkey is closer to the
 *                 query's in dist_e (ties to the left) until r (r1) positions
 *                 are taken.  Applies to both layers.
 *  pass_pairs     most (query, cluster) pairs per MFMA pass of the rerank:
 *                 16, 32, 64, 128, or 0 (32, 64 or 128 as that expected
 *                 overlap is at most 16, at most 48, or more); 64-row tiles
 *                 take at most 64, 128-row tiles at most 32.  A tile overlapped by P pairs is
 *                 streamed ceil(P / pass_pairs) times.  Results are identical. */
typedef struct {
  int32_t r1;
  int32_t precision;
  int32_t shortlist_mult;
  int32_t persistent;
  int32_t tile_rows;
  int32_t l1_dense;
  int32_t grid_mult;
  int32_t pass_pairs;
  int32_t expand_bits;
  int32_t reserved[7];
} lider_search_opts;

/* Optional device outputs of the intermediate search state, for parity checks.
 * Each pointer may be NULL.  H = the index's n_arrays.
 *  qdigits_dev [nq x 2Hm] int32  query digits (layer-1 sets of arrays 0..H-1,
 *                                then the layer-2 sets)
 *  l1_dev      [nq x H x 3] int64 per array: layer-1 predicted location,
 *                                window start, length
 *  routed_dev  [nq x c] int32    routed cluster ids (order unspecified, -1 pad)
 *  pairs_dev   [nq x c x H x 3] int64 per routed cluster (same order) and
 *                                array: predicted location, window start,
 *                                window length */
typedef struct {
  int32_t* qdigits_dev;
  int64_t* l1_dev;
  int32_t* routed_dev;
  int64_t* pairs_dev;
} lider_search_debug;

/* Bytes of device workspace lider_search / lider_search_ex need for a batch.
 * Non-decreasing in nq and in k (all else equal): a workspace sized for the
 * largest batch and k serves every smaller one.  Returns 0 for invalid
 * arguments. */
size_t lider_search_workspace(const lider_index* index, int64_t nq, int32_t k, int32_t c,
                              int32_t r, const lider_search_opts* opts);

/* Batched search (Section 3.3.2): queries_dev [nq x d] fp32.  For each query:
 * hash digits of both layers; the centroids retriever's key, RMI location and
 * window of r1 centroids, scored by inner product, top c clusters; in each
 * routed cluster the in-cluster retriever's key, RMI location and window of r
 * rows; exact inner-product scores of all window rows; top k over the union.
 * With H hashkey arrays every array contributes its own window in both layers
 * and the candidates of a core model are the union of its H windows.
 * Outputs ids_dev [nq x k] int64 (original row ids) and scores_dev [nq x k]
 * fp32, each row sorted by score descending, ties by smaller id, padded with
 * id -1 / score -inf.  ws_dev must hold lider_search_workspace(...) bytes (256-
 * byte aligned).  Asynchronous on `stream`: nothing is allocated, nothing is
 * synchronised, no host read-back.  k in 1..LIDER_MAX_K, c in
 * 1..min(LIDER_MAX_C, n_clusters), r >= 1, nq >= 0 (0 is a no-op).
 * A query holding a NaN or an infinity gets ids that are -1 or rows of the
 * corpus (which ones is unspecified); the other queries of the batch are
 * unaffected.
 * Safe to call concurrently on different streams with separate workspaces. */
int lider_search(const lider_index* index, const float* queries_dev, int64_t nq, int32_t k,
                 int32_t c, int32_t r, int64_t* ids_dev, float* scores_dev, void* ws_dev,
                 size_t ws_bytes, void* stream);

/* lider_search with options (NULL = defaults) and optional debug outputs. */
int lider_search_ex(const lider_index* index, const float* queries_dev, int64_t nq, int32_t k,
                    int32_t c, int32_t r, int64_t* ids_dev, float* scores_dev, void* ws_dev,
                    size_t ws_bytes, void* stream, const lider_search_opts* opts,
                    const lider_search_debug* debug);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the search of
 * lider_search_ex (same arguments, results bit-identical) with its workspace in
 * a fixed array inside the library instead of a caller's buffer.  No
 * allocation of any kind, no synchronisation.  The array holds
 * lider_noalloc_scratch_bytes() bytes (64 MiB) on every GPU the library runs
 * on, until the process ends; a batch whose lider_search_workspace exceeds it
 * is rejected with LIDER_EINVAL before anything is enqueued.  Every call on a
 * GPU uses that GPU's one array: calls that overlap on one GPU (on different
 * streams, or from several threads without ordering) race and are not
 * allowed; consecutive calls on one stream are fine.  The first call on a
 * device resolves the array's device address (once per device). */
int lider_search_noalloc(const lider_index* index, const float* queries_dev, int64_t nq,
                         int32_t k, int32_t c, int32_t r, int64_t* ids_dev, float* scores_dev,
                         void* stream, const lider_search_opts* opts);

/* Size in bytes of lider_search_noalloc's fixed workspace. */
size_t lider_noalloc_scratch_bytes(void);

/* ---------------------------------------------------------------- inspection */

typedef struct {
  int64_t n;
  int32_t d, n_clusters, m, rmi_fanout, rmi_fanout_l1;
  int32_t kmeans_iters_run; /* Lloyd assignments executed (0 if given) */
  int64_t max_cluster;      /* largest cluster size */
  double w;
  int32_t storage, centroid_storage;
  int32_t n_arrays;         /* hashkey arrays per core model */
  int32_t hash_kind;        /* LIDER_HASH_E2LSH or LIDER_HASH_SIGN */
} lider_info;

int lider_get_info(const lider_index* index, lider_info* out);

/* Exportable index arrays (host copies, synchronous).  Per-array tables are
 * array-major (array h's block follows array h-1's); H = n_arrays.  The
 * reordered corpus and every "sorted position" of a search are array 0's. */
typedef enum {
  LIDER_X_CENTROIDS = 0,  /* [C x d] fp32, cluster-id order */
  LIDER_X_ASSIGN = 1,     /* [n] int32 cluster of each original row */
  LIDER_X_OFFSETS = 2,    /* [C+1] int64 first sorted position of each cluster */
  LIDER_X_PERM = 3,       /* [H x n] int64 sorted position -> original row id */
  LIDER_X_KEYS = 4,       /* [H x n] uint64 key at each sorted position */
  LIDER_X_DIGITS = 5,     /* [H x n x m] int32 layer-2 digits per original row */
  LIDER_X_L1_ORDER = 6,   /* [H x C] int64 layer-1 sorted position -> cluster id */
  LIDER_X_L1_KEYS = 7,    /* [H x C] uint64 */
  LIDER_X_L1_DIGITS = 8,  /* [H x C x m] int32 layer-1 digits per cluster id */
  LIDER_X_MODEL_INT = 9,  /* [H x (C+1) x 3] int64: L, m_eff, F; model C = layer 1 */
  LIDER_X_MODEL_BOX = 10, /* [H x (C+1) x 2m] int32: mins[m], maxs[m] */
  LIDER_X_MODEL_KEY = 11, /* [H x (C+1) x 2] uint64: kmin, kmax */
  LIDER_X_MODEL_DBL = 12, /* [H x (C+1) x 3] double: scale, root slope, root intercept */
  LIDER_X_LEAVES = 13,    /* [H x (C*F2 + F1)] x 2 double: leaf slope, intercept */
  LIDER_X_LEAF_ERR = 14,  /* [H x (C*F2 + F1)] x 2 int32: min and max (true - predicted) */
  LIDER_X_REORDERED = 15  /* [n x d] fp32 corpus in sorted order */
} lider_export_what;

/* Bytes of one export (0 if unknown / not present). */
size_t lider_export_bytes(const lider_index* index, int32_t what);
/* Copy one array to host memory dst_host of dst_bytes >= lider_export_bytes. */
int lider_export(const lider_index* index, int32_t what, void* dst_host, size_t dst_bytes);

/* ------------------------------------------------------------ persistence */

/* Write the whole index (every device array and the parameters) to the file
 * `path` (created or truncated), synchronously: the parameters, then each
 * array as a tagged, sized section in a fixed order (the format is this
 * library's own, for the same byte order).  A corpus of n x d fp32 takes
 * 4 n d bytes plus the per-array tables.  Errors: EINVAL, EIO, EDEVICE. */
int lider_save(const lider_index* index, const char* path);

/* Read an index written by lider_save onto the current HIP device: allocate
 * its device memory, copy every section, rebuild the host-side tables.  The
 * loaded index searches bit-identically to the saved one.  Runs on `stream`
 * and synchronises it.  Errors: EINVAL (NULL argument), EIO (missing or
 * truncated file, wrong format or version, section sizes that do not match
 * the parameters), ENOMEM, EDEVICE; on error *out is NULL. */
int lider_load(const char* path, void* stream, lider_index** out);

/* ------------------------------------------------------- stand-alone kernels */

/* E2LSH digits (Section 4): out_dev[r*nh + i] = floor((A[i].X[r] + b[i]) / w)
 * for X_dev [n x d], A_dev [nh x d], b_dev [nh] (all fp32, device), nh in 1..512.
 * Projections run on FP64 MFMA over the exact fp32 x fp32 products; values
 * within the rounding-error band of a bucket edge are recomputed by the
 * sequential FP64 sum, so the digits equal the FP64 definition exactly.
 * Allocates small temporary device buffers (row-norm bounds of A, a status
 * word); synchronises `stream`.  Errors: EINVAL, ENOMEM, EDEVICE, ERANGE (a
 * digit outside int32). */
int lider_hash(const float* X_dev, int64_t n, int32_t d, const float* A_dev, const float* b_dev,
               int32_t nh, double w, int32_t* out_dev, void* stream);

/* One k-means assignment step (Section 3.2): assign_dev[i] = argmin_j
 * ||X[i] - cent[j]||^2 decided in FP64 (ties to the smaller j); fp32 MFMA
 * distances, FP64 recompute where the rounding-error bands of the two best
 * overlap.  X_dev [n x d], cent_dev [C x d].  Allocates temporaries;
 * synchronises `stream`. */
int lider_kmeans_assign(const float* X_dev, int64_t n, int32_t d, const float* cent_dev,
                        int32_t C, int32_t* assign_dev, void* stream);

/* ------------------------------------------------------------- profiling */

/* Search stages timed by lider_profile_*: 0 query hashing, 1 layer-1 location
 * and routing, 2 layer-2 locations and the per-cluster work list, 3 rerank
 * (the window scoring kernel), 4 top-k selection (and the precision form's
 * fp32 shortlist rerank). */
#define LIDER_NSTAGES 5

/* Start timing the next max_calls (1..4096) lider_search / lider_search_ex
 * calls made on this thread: HIP events are created now and recorded on each
 * call's stream around every stage (no allocation in the searches). */
int lider_profile_begin(int32_t max_calls);

/* Wait for the recorded events, return the summed device time of each stage
 * in stage_ms[LIDER_NSTAGES] (milliseconds) and the number of timed calls,
 * release the events and stop timing. */
int lider_profile_end(double* stage_ms, int32_t* calls);

/* Test hook: the next lider_search / lider_search_ex call on this thread fails
 * with `status` before enqueuing anything (0 clears the hook). */
void lider_debug_fail_next(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* LIDER_H */
