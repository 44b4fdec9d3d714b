/*
 * patchwork.h -- C-ABI of libpatchwork.so: real schemes of T-curves on
 * MI355X (gfx950).
 *
 * The library evaluates Algorithm 1 of "Fast Isotopy Computation for
 * T-Curves" (Sec. 2) for very many pairs (T, sigma) at once: T is a
 * unimodular triangulation of d*Delta_2 given by its edge list (Sec. 2),
 * sigma : A -> GF(2) a sign distribution on its lattice points.  Each
 * evaluation reflects the signs into the four quadrant copies (eq. (signs)),
 * glues the copies into RP^2 by identifying antipodal boundary points,
 * merges same-sign components into regions, builds the region adjacency
 * tree, roots it (Alg. 1: odd d -> the region with a self-loop, even d ->
 * the region whose components form an odd antipodal cycle) and returns a
 * canonical code of the rooted tree.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice points: A = {(i,j) : i,j >= 0, i+j <= d} (eq. (lattice)), |A| =
 *   (d+1)(d+2)/2, numbered k(i,j) = j(d+1) - j(j-1)/2 + i.
 * Sign masks: bit k of a mask is sigma(p_k); 0 means '+' (the coefficient
 *   sign is (-1)^sigma, Thm. 1).  A mask is stored in the narrowest of
 *   uint32 (|A| <= 32, d <= 6), uint64 (|A| <= 64, d <= 9) or two uint64
 *   little-endian words (d >= 10); pw_mask_bytes() returns the width.  Bits
 *   >= |A| are ignored.  Flipping every sign (bit 0 included) leaves the
 *   scheme unchanged.
 * Scheme code: 128 bits as two uint64 (lo, hi).  For a node v of the rooted
 *   region tree, c(v) = '1' . concat(c(children), sorted descending with
 *   '1' > '0') . '0'; W is the concatenation of the sorted codes of the
 *   root's children; code = 2^|W| + W (first character of W most
 *   significant); bit 127 is set iff d is odd (the pseudo-line J).  Valid
 *   codes are never 0; 0 marks an evaluation that failed an internal
 *   consistency check (see pw_tri_errors).  The number of ovals is
 *   (bit length of the code without bit 127 - 1) / 2.
 * Memory: every pointer named d_* is device memory owned by the caller and
 *   must stay valid until the stream has finished the call.  Handles
 *   (pw_tri_t, pw_hist_t) are owned by the library; create and destroy them
 *   explicitly.  Other pointers are host memory, read before the call
 *   returns.
 * Streams: every compute call is asynchronous on the hipStream_t it is
 *   given (0 = the null stream).  A handle must not be used from two
 *   streams at once without synchronisation.
 * Errors: every call returns pw_status (PW_OK = 0 or a negative code) and
 *   never throws; pw_last_error() returns a thread-local message for the
 *   last failing call.
 */
#ifndef PATCHWORK_H
#define PATCHWORK_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pw_status;

#define PW_OK 0
#define PW_ERR_ARG (-1)       /* bad argument: null pointer, size, degree     */
#define PW_ERR_TRI (-2)       /* the edge list is not a unimodular triangulation */
#define PW_ERR_HIP (-3)       /* a HIP runtime call failed                      */
#define PW_ERR_RANGE (-4)     /* enumeration range beyond 2^(free bits)         */
#define PW_ERR_HIST_FULL (-5) /* a histogram ran out of slots (sticky)          */
#define PW_ERR_INTERNAL (-6)  /* a device-side consistency check failed         */

typedef struct pw_tri *pw_tri_t;
typedef struct pw_hist *pw_hist_t;

/* Thread-local message describing the last failing call ("" if none). */
const char *pw_last_error(void);

/* Library version as an integer (major*10000 + minor*100 + patch). */
int32_t pw_version(void);

/* Bytes per sign mask for degree d (4, 8 or 16), or PW_ERR_ARG. */
int32_t pw_mask_bytes(int32_t d);

/*
 * Create a triangulation handle (Sec. 2: T is represented by its edge list).
 *   d         degree, 1 <= d <= 12.
 *   edges_ij  host array of n_edges rows (i0, j0, i1, j1), endpoints in A.
 *   n_edges   must equal |A| + d^2 - 1.
 *   out       receives the handle.
 * Validation: endpoints in A, edges primitive and distinct, exactly d^2
 * unimodular (area 1/2) triangles among the edge-graph 3-cliques, every
 * boundary edge in one triangle and every interior edge in two triangles on
 * opposite sides.  Regularity is not required (proof of Thm. 2: the
 * computation needs neither regularity nor, beyond the full point set,
 * unimodularity).  Builds the reflected diamond A<>, E(T<>) and the 2d
 * antipodal boundary pairs, and uploads them to the current device.
 * Errors: PW_ERR_ARG, PW_ERR_TRI, PW_ERR_HIP.
 */
pw_status pw_tri_create(int32_t d, const int16_t *edges_ij, int32_t n_edges, pw_tri_t *out);

pw_status pw_tri_destroy(pw_tri_t tri);

/* Sizes of a handle: d, |A|, |A<>| = 2d^2+2d+1, |E(T<>)| = 6d^2+2d (Table 1),
 * number of antipodal pairs (2d).  Any output pointer may be NULL. */
pw_status pw_tri_info(pw_tri_t tri, int32_t *d, int32_t *n_points, int32_t *n_vertices,
                      int32_t *n_diamond_edges, int32_t *n_antipodal_pairs);

/* Synchronise the device and return (then clear) the handle's sticky
 * device-side error flags: bit 0 = more regions than Harnack's bound allows
 * (Sec. 2), bit 1 = no unique root, bit 2 = the adjacency graph is not a
 * tree, bit 3 = a self-loop for even d.  0 means every evaluation passed. */
pw_status pw_tri_errors(pw_tri_t tri, uint32_t *flags);

/*
 * Build kernels specialised to this triangulation (d <= 9): the walk of
 * Alg. 1 over its diamond (Sec. 2) is written out as straight-line code with
 * the vertex, neighbour and antipodal-pair indices as literals, compiled with
 * hipRTC for gfx950 and loaded on the current device.  Afterwards
 * patchwork_scheme_batch / _histogram / _enumerate_range on this handle use
 * them; results are identical to the generic kernels.  Takes seconds (a
 * compile; the code object is kept per generated source for the life of the
 * process, so an equal triangulation loads it without compiling again);
 * idempotent.  Errors: PW_ERR_ARG (d > 9), PW_ERR_HIP (compile or
 * load failed; the handle keeps using the generic kernels).
 */
pw_status pw_tri_specialize(pw_tri_t tri);

/* Copy the handle's program (the reflected diamond in the layout the
 * kernels walk: per diamond vertex its lattice point, reflection parity and
 * earlier neighbours, then the 2d antipodal pairs; Alg. 1, first steps) into
 * a host buffer of cap words; *n_words receives its length (words may be
 * NULL to query it).  Host memory only; PW_ERR_ARG if cap is too small. */
pw_status pw_tri_program(pw_tri_t tri, uint32_t *words, int32_t cap, int32_t *n_words);

/* Copy the handle's group program for G = 2 or 4 lanes per mask (one block
 * of the reflected diamond, Sec. 2: the half y >= 0 or the quadrant
 * x, y >= 0, with its earlier neighbours, then the glues that join the
 * copies of an axis point in two blocks and the 2d antipodal pairs, in
 * group indices v * G + q) into a host buffer of cap words, as
 * pw_tri_program.  Degrees 8..12 only.  Errors: PW_ERR_ARG (other G or
 * degree, cap too small). */
pw_status pw_tri_group_program(pw_tri_t tri, int32_t G, uint32_t *words, int32_t cap, int32_t *n_words);

/* ------------------------------------------------------------------------
 * Symmetries of the search space (Sec. 3, Table 1).  Host calls; no device
 * work.
 *
 * S3 acts on d*Delta_2 by permuting the barycentric coordinates
 * (i, j, d-i-j); permutation k in 0..5 is the k-th of (0,1,2) (0,2,1)
 * (1,0,2) (1,2,0) (2,0,1) (2,1,0) in this order, sending (i, j) to
 * (b[P0], b[P1]) with b = (i, j, d-i-j).  It maps a triangulation T and a
 * sign distribution sigma to (pi T, sigma o pi^-1), which have the same
 * real scheme, so one member of each orbit of triangulations (6 members, 3
 * for those fixed by a transposition, 1 for the fully symmetric) stands for
 * all.  (Z/2)^3 acts on sign distributions by sigma -> sigma + a + b i + c j
 * (mod 2), freely and without changing the scheme: one representative per
 * class covers 8 distributions.
 * ---------------------------------------------------------------------- */

/* Canonical member of the S3 orbit of T: the image whose edge list (each
 * edge with its endpoints in point-index order, edges sorted by the point
 * indices of their endpoints) is lexicographically least, written to
 * out_edges (host, n_edges x 4, in that order; may be NULL); *perm_index
 * receives a permutation k that maps T to it and *stabilizer the number of
 * permutations fixing T (1, 2, 3 or 6; the orbit has 6 / stabilizer
 * members).  T is validated as in pw_tri_create (PW_ERR_TRI). */
pw_status pw_tri_canonical(int32_t d, const int16_t *edges_ij, int32_t n_edges, int16_t *out_edges,
                           int32_t *perm_index, int32_t *stabilizer);

/* out[k] = index of the image under permutation perm_index of lattice point
 * k, for k < |A| (host array).  A sign mask maps to the permuted
 * triangulation's by moving bit k to bit out[k]. */
pw_status pw_point_map(int32_t d, int32_t perm_index, int32_t *out);

/* The fixed_zero_bits (two uint64 words) that make
 * patchwork_scheme_enumerate_range visit one representative of each
 * (Z/2)^3 class: sigma = '+' at (0,0) and at two points of distinct nonzero
 * parity classes (i mod 2, j mod 2), taken from lattice point 10 on when
 * the degree allows (so points 1..9 stay free and the sweep kernel with a
 * shared snapshot applies).  The free bits number |A| - 3.  d >= 2. */
pw_status pw_class_fixed_bits(int32_t d, uint64_t out[2]);

/* The source text pw_tri_specialize compiles for the triangulation given
 * by (d, edges_ij, n_edges) (validated as in pw_tri_create), into a host
 * buffer of cap bytes, NUL-terminated and truncated to fit; *len receives
 * the full length.  Needs no GPU. */
pw_status pw_jit_source(int32_t d, const int16_t *edges_ij, int32_t n_edges, char *buf, int64_t cap,
                        int64_t *len);

/* Compile that source with hipRTC for gfx950 without loading it (needs no
 * GPU); *code_bytes receives the code object size. */
pw_status pw_jit_compile(int32_t d, const int16_t *edges_ij, int32_t n_edges, int64_t *code_bytes);

/*
 * Codes of n sign masks (Alg. 1 for each pair (T, sigma_k)).
 *   d_masks  n masks of pw_mask_bytes(d) bytes each, contiguous.
 *   d_codes  n x 2 uint64 (lo, hi) written in input order, 16-byte aligned
 *            (each code is one 16-byte store).
 * n = 0 is a no-op; n < 0 or a misaligned d_codes is PW_ERR_ARG.
 */
pw_status patchwork_scheme_batch(pw_tri_t tri, const void *d_masks, int64_t n, uint64_t *d_codes,
                                 hipStream_t stream);

/*
 * Histogram handle: an open-addressing table code -> (count, witness) in
 * device memory, capacity a power of two >= the number of distinct codes
 * expected.  pw_hist_reset clears it asynchronously.  pw_hist_read
 * synchronises the device, merges and sorts the entries by code (as 128-bit
 * unsigned integers) and copies at most `capacity` of them to host arrays
 * codes (n x 2 uint64), counts (n), witness (n); n_used receives the number
 * of distinct codes.  It returns PW_ERR_HIST_FULL if any insert found no
 * free slot since the last reset (the table is then incomplete).
 */
pw_status pw_hist_create(int32_t capacity, pw_hist_t *out);
pw_status pw_hist_reset(pw_hist_t hist, hipStream_t stream);
pw_status pw_hist_read(pw_hist_t hist, uint64_t *codes, uint64_t *counts, uint64_t *witness,
                       int32_t capacity, int32_t *n_used);
pw_status pw_hist_destroy(pw_hist_t hist);

/*
 * Codes and histogram of the same n masks in one pass (each mask evaluated
 * once): d_codes as in patchwork_scheme_batch, `hist` as in
 * patchwork_scheme_histogram (accumulates; witness = smallest index_base +
 * k).  Sec. 3: a sweep wants both the scheme of every sign distribution and
 * the per-triangulation distribution.  Errors as those two calls.
 */
pw_status patchwork_scheme_codes_histogram(pw_tri_t tri, const void *d_masks, int64_t n, uint64_t index_base,
                                           uint64_t *d_codes, pw_hist_t hist, hipStream_t stream);

/*
 * Histogram of the codes of n masks (the per-triangulation distribution of
 * schemes; Sec. 3, exhaustive search mode).  Accumulates into `hist`
 * without resetting it.  The witness of a code is the smallest
 * index_base + k over the masks d_masks[k] that produced it.
 */
pw_status patchwork_scheme_histogram(pw_tri_t tri, const void *d_masks, int64_t n, uint64_t index_base,
                                     pw_hist_t hist, hipStream_t stream);

/*
 * Histogram over an index range of generated masks (Sec. 3: sweep all sign
 * distributions of one triangulation).  The free bits are the bits < |A|
 * not set in fixed_zero_bits (two uint64 words, host memory); mask(k) puts
 * the bits of first+k, lowest first, into the free bit positions and leaves
 * the fixed bits 0.  With fixed_zero_bits = {1, 0} (sigma(0,0) = '+') the
 * range [0, 2^(|A|-1)) covers every scheme once per global sign flip; with
 * the three points (0,0), (1,0), (0,1) fixed it visits one representative of
 * each (Z/2)^3 class (Sec. 3, Table 1).  The witness of a code is the
 * smallest index first+k that produced it.  The free positions may form at
 * most 4 contiguous runs.  Errors: PW_ERR_RANGE if first+count exceeds
 * 2^(number of free bits), PW_ERR_ARG for more than 4 runs.
 */
pw_status patchwork_scheme_enumerate_range(pw_tri_t tri, uint64_t first, uint64_t count,
                                           const uint64_t fixed_zero_bits[2], pw_hist_t hist,
                                           hipStream_t stream);

/*
 * The same histogram as patchwork_scheme_enumerate_range(first, count), as
 * a chunked sweep: ceil(count / chunk) launches of at most `chunk` masks
 * each, captured once into a HIP graph and launched as one graph on
 * `stream` (a sweep issued in many short launches pays one host submission
 * instead of one per launch; Sec. 3 exhaustive search at scale).  The
 * triangulation handle owns the graph and keeps it for the last argument
 * set (first, count, chunk, fixed bits, hist): calling again with the same
 * arguments launches the kept graph again (the histogram accumulates once
 * more), other arguments capture a new one.  Capture happens on a stream of
 * the handle's own, so `stream` may be the default stream.  The kept graph
 * names its histogram by a serial number that pw_hist_create never reuses, so
 * a histogram created after another was destroyed (even at the same address)
 * gets a new capture; a histogram must not be destroyed while a launch of
 * the graph may still run on it.  Errors: as
 * patchwork_scheme_enumerate_range, plus PW_ERR_ARG for chunk == 0 or more
 * than 2^16 launches, PW_ERR_HIP if the capture fails.  Not for concurrent
 * use of one handle from several threads.
 */
pw_status patchwork_scheme_sweep_graph(pw_tri_t tri, uint64_t first, uint64_t count, uint64_t chunk,
                                       const uint64_t fixed_zero_bits[2], pw_hist_t hist, hipStream_t stream);

/*
 * Many triangulations of uneven degree in one call (Sec. 3: the second
 * search mode sweeps many triangulations; kernel dispatch and histogram
 * aggregation are the costs at scale).
 *   tris      n_tris handles (host array), any mix of degrees.
 *   d_masks   one array of 128-bit masks (two uint64 per mask, whatever the
 *             degree); triangulation t owns masks [offsets[t], offsets[t+1]).
 *   offsets   host array of n_tris + 1 non-decreasing indices.
 *   hists     host array of n_tris histogram handles, or NULL; the witness
 *             of a code is its smallest global mask index.
 *   d_codes   NULL, or n x 2 uint64 codes written at the masks' positions
 *             (16-byte aligned).
 *   cfg       NULL for the defaults (4096 masks per item, one wave per
 *             block, blocks per CU as LDS and registers allow, lane groups
 *             PW_MULTI_DEFAULT_LANE_GROUPS), or the tuned launch shape:
 *             masks per work item, waves per block (lowered until a block's
 *             LDS for the largest degree of its class fits in 160 KiB),
 *             blocks per CU (0 = as many as LDS and registers allow), and
 *             lanes per mask for each degree: bits 2d..2d+1 of lane_groups
 *             are 0 (one lane per mask), 1 (two lanes: the halves y >= 0 and
 *             y <= 0 of the reflected diamond, Sec. 2) or 2 (four lanes: the
 *             four reflected copies of the triangulation); 1 and 2 are
 *             allowed for degrees 8..12 only (PW_ERR_ARG otherwise).  The
 *             codes do not depend on the shape.  The library reads no tuning cache itself: the tuned
 *             shapes are kept per degree mix by the Python layer (tune.py,
 *             in tune_cache_gfx950.json beside it, or the file named by the
 *             PW_TUNE environment variable); a C caller passes the shape it
 *             wants here.
 * Degrees are grouped into LDS classes (those whose per-wave areas allow
 * the same number of resident blocks per CU); each class is one persistent
 * launch, sized for its largest degree, and the launches run back to back
 * on `stream`.  Within a launch, work items (chunks of one triangulation's
 * masks) are taken from an atomic queue in decreasing order of cost.  The
 * call returns after the last launch has finished (its device tables are
 * reused by the next call).
 */
typedef struct {
  int32_t chunk;
  int32_t waves_per_block;
  int32_t blocks_per_cu;
  uint32_t lane_groups;
} pw_multi_config;

/* Lane groups used when cfg is NULL: four lanes per mask for degrees 11 and 12. */
#define PW_MULTI_DEFAULT_LANE_GROUPS ((2u << 22) | (2u << 24))

pw_status patchwork_scheme_batch_multi(const pw_tri_t *tris, int32_t n_tris, const void *d_masks,
                                       const int64_t *offsets, const pw_hist_t *hists, uint64_t *d_codes,
                                       const pw_multi_config *cfg, hipStream_t stream);

/*
 * patchwork_scheme_batch_multi for callers that cannot allocate device
 * memory (code that must not call hipMalloc: tight serving loops, harnesses
 * that forbid allocation).  Same arguments, launches and results as
 * patchwork_scheme_batch_multi; its descriptor and work-item tables, ticket
 * counter and overflow list live in one fixed device array of the library
 * (about 7.4 MiB per GPU, held from the first call on that GPU until the
 * process ends) instead of buffers the library allocates.  It calls no
 * hipMalloc or hipFree.  Limits: n_tris <= PW_NOALLOC_MAX_TRIS; at most
 * PW_NOALLOC_MAX_ITEMS work items (sum over t of ceil(masks of t / chunk));
 * at most PW_NOALLOC_MAX_OVERFLOW masks of degree >= 10 with more than 31
 * ovals per call.  Beyond the first two: PW_ERR_ARG before anything is
 * launched; beyond the third: PW_ERR_INTERNAL (split the call).  Every call
 * on one GPU uses that GPU's array and keeps nothing in it between calls
 * (the counters are cleared at the start of each).  Calls that overlapped
 * on one GPU would race on it, so the library serialises calls from the
 * threads of a process, and a call returns only after its launches have
 * finished; after an error return, synchronise `stream` before the next
 * call, since a launch made before the error may still be running.
 */
#define PW_NOALLOC_MAX_TRIS 4096
#define PW_NOALLOC_MAX_ITEMS 262144
#define PW_NOALLOC_MAX_OVERFLOW 65536

pw_status patchwork_scheme_batch_multi_noalloc(const pw_tri_t *tris, int32_t n_tris, const void *d_masks,
                                               const int64_t *offsets, const pw_hist_t *hists, uint64_t *d_codes,
                                               const pw_multi_config *cfg, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Search over triangulations (Sec. 3: the second search mode checks many
 * (symmetric) triangulations against a few witness sign distributions;
 * simulated annealing over triangulations optimises the number of distinct
 * types or a target (p, n) count).
 *
 * A triangulation of d*Delta_2, d <= 9, lives in device memory as 64
 * uint64 adjacency rows: bit q of row p is set iff lattice points p and q
 * (numbered as for sign masks) are joined by an edge; rows >= |A| are 0.
 * A batch of n triangulations is n x 64 uint64, contiguous.  Every buffer
 * named d_* is device memory owned by the caller; calls are asynchronous
 * on `stream`.
 * ---------------------------------------------------------------------- */

/* Host: the adjacency rows (64 uint64, host) of an edge list, validated as
 * in pw_tri_create.  d <= 9.  Errors: PW_ERR_ARG, PW_ERR_TRI. */
pw_status pw_adjacency_from_edges(int32_t d, const int16_t *edges_ij, int32_t n_edges, uint64_t *rows);

/* Host: the edge list (i0, j0, i1, j1 rows, endpoints in increasing point
 * order, edges in increasing order) of 64 adjacency rows, into edges_ij of
 * cap rows; *n_edges receives the count (edges_ij may be NULL to query).
 * PW_ERR_TRI for an asymmetric adjacency or bits beyond |A|. */
pw_status pw_edges_from_adjacency(int32_t d, const uint64_t *rows, int16_t *edges_ij, int32_t cap,
                                  int32_t *n_edges);

/*
 * Random walks in the flip graph, in place: `steps` proposed moves on each
 * of n_tris triangulations (one wavefront each).  A flip replaces an
 * interior edge ab, whose two unimodular triangles abc, abe form a
 * parallelogram (c + e = a + b), by the diagonal ce (the flips connect all
 * unimodular triangulations of d*Delta_2).  Move s of triangulation w draws
 * r1 = F(seed ^ F(w * 0x100000001B3 + 2 (step0 + s))) and r2 the same with
 * + 1 (F = the SplitMix64 finaliser): a = r1 mod |A|, b = the
 * (r2 mod deg a)-th neighbour of a in increasing point order, and ab is
 * flipped if it can be.  symmetric != 0 keeps (i, j) -> (j, i) symmetry
 * (the input must be symmetric): an edge mapped to itself is flipped
 * alone; otherwise ab and its mirror image are flipped together when both
 * can be and their quadrilaterals share no triangle; other moves change
 * nothing.  d_moves (n_tris uint32, or NULL) is incremented by the number of
 * moves made.  d <= 9.
 */
pw_status pw_flip_walk(int32_t d, uint64_t *d_adj, int64_t n_tris, int32_t steps, int32_t symmetric, uint64_t seed,
                       uint64_t step0, uint32_t *d_moves, hipStream_t stream);

/* Words of one triangulation's program (the layout of pw_tri_program):
 * |A<>| + |E(T<>)| + 2d. */
int32_t pw_program_words(int32_t d);

/* The program of each of n_tris triangulations (d_adj) built on the device
 * into d_progs (n_tris x pw_program_words(d) uint32), word for word what
 * pw_tri_create builds for the same edge list.  d_bad[t] (uint32) becomes
 * non-zero if triangulation t's program could not be built (its adjacency
 * is not a unimodular triangulation); its program is then unusable. d <= 9. */
pw_status pw_build_programs(int32_t d, const uint64_t *d_adj, int64_t n_tris, uint32_t *d_progs, uint32_t *d_bad,
                            hipStream_t stream);

/*
 * Every triangulation of a batch against every witness (Alg. 1 for each of
 * n_tris x n_w pairs): d_progs as built by pw_build_programs (any degree
 * 1..12), d_masks n_w witnesses of two uint64 words each.  The code of
 * (t, w) goes to d_codes[t * n_w + w] (n_tris x n_w x 2 uint64, 16-byte
 * aligned, or NULL) and/or into `hist` (or NULL) with witness t * n_w + w.
 * d_err (one uint32) accumulates the device consistency flags of
 * pw_tri_errors.
 */
pw_status patchwork_scheme_programs(int32_t d, const uint32_t *d_progs, int64_t n_tris, const uint64_t *d_masks,
                                    int64_t n_w, uint64_t *d_codes, pw_hist_t hist, uint32_t *d_err,
                                    hipStream_t stream);

/* Score of each triangulation over its n_w codes d_codes[t * n_w ..], as
 * float: mode 0 = number of distinct codes (the number of types it
 * realises on those witnesses), mode 1 = number of codes whose scheme has
 * (p, n) = (target_p, target_n) (p ovals at odd depth, outermost = depth 1;
 * n at even depth), mode 2 = number of distinct codes whose low word is not
 * in d_known (n_known uint64 in increasing order: the types found so far).
 * Codes 0 count for nothing.  d <= 9 (a code's low word then holds all of
 * it but the J bit), n_w <= 8192. */
pw_status pw_tri_objective(int32_t d, const uint64_t *d_codes, int64_t n_tris, int32_t n_w, int32_t mode,
                           int32_t target_p, int32_t target_n, const uint64_t *d_known, int32_t n_known,
                           float *d_score, hipStream_t stream);

/*
 * Metropolis step of simulated annealing over triangulations (maximising
 * the score), for n_chains chains of adjacency rows: the proposal d_prop
 * (scored d_score_prop) replaces d_cur (d_score_cur) if it scores at least
 * as high, or else if u < d_accept[k - 1], k = score_cur - score_prop (the
 * scores are whole numbers), u = the top 24 bits of
 * F(seed ^ F(chain * 0x100000001B3 + step)); d_accept holds
 * floor(2^24 exp(-k / temperature)) for k = 1 .. n_accept, computed by the
 * caller (0 beyond).  Then d_prop is set equal to d_cur.  d_best /
 * d_score_best keep each chain's best state; d_n_accepted[chain] counts
 * accepted proposals.
 */
pw_status pw_anneal_accept(uint64_t *d_cur, uint64_t *d_prop, float *d_score_cur, const float *d_score_prop,
                           uint64_t *d_best, float *d_score_best, int64_t n_chains, const uint32_t *d_accept,
                           int32_t n_accept, uint64_t seed, uint64_t step, uint32_t *d_n_accepted,
                           hipStream_t stream);

/* ------------------------------------------------------------------------
 * Learned proposal of sign distributions.
 *
 * Not a step of Alg. 1: the paper finds rare schemes by searching over
 * triangulations and curated pools of witnesses (Sec. 3).  These calls build
 * a proposal generator for that search: a multilayer perceptron
 * (|A| -> 512 -> 512 -> 64, ReLU) trained on masks labelled by the exact
 * kernels above, used to rank mutated witnesses; every proposal it keeps is
 * then judged by patchwork_scheme_batch / _histogram.  All buffers are
 * device memory owned by the caller; every call is asynchronous on `stream`
 * and returns PW_ERR_ARG (nothing launched) on bad sizes or null buffers.
 * bfloat16 values are uint16_t bit patterns (upper half of an IEEE binary32,
 * rounded to nearest even).  Masks here are always two uint64 per mask.
 * ---------------------------------------------------------------------- */

/*
 * C = A B (+ bias[n]) (ReLU) (* [gate > 0]) on gfx950 BF16 matrix cores with
 * FP32 accumulation.  Element (m, k) of A is A[m * a_m + k * a_k], element
 * (k, n) of B is B[k * b_k + n * b_n] (so one call serves X W, dY W^T and
 * X^T dY); gate (M x N, row stride g_m) and bias (N floats) may be NULL.
 * Output row stride c_m; C32 (fp32) and/or C16 (bf16), at least one;
 * accumulate != 0 adds into C32.  colsum (N floats, or NULL) receives
 * colsum[n] += sum over m of the final C[m][n] (after the epilogue, before
 * bf16 rounding; FP32 atomics, in no fixed order) -- the bias gradient of a
 * backward product.  M and N must be multiples of 64, K of 32.
 */
pw_status pw_mlp_gemm(const uint16_t *A, int64_t a_m, int64_t a_k, const uint16_t *B, int64_t b_k, int64_t b_n,
                      int32_t M, int32_t N, int32_t K, const float *bias, const uint16_t *gate, int64_t g_m,
                      int32_t relu, float *C32, uint16_t *C16, int64_t c_m, int32_t accumulate, float *colsum,
                      hipStream_t stream);

/*
 * Network input: X[k][j] = +1 for sign '+' (bit j of mask k clear), -1 for
 * '-', j < n_bits (bits in the point order of eq. (signs)); 0 in the padding
 * columns n_bits <= j < width.  X is n x width bf16.
 */
pw_status pw_mlp_encode(const uint64_t *masks, int64_t n, int32_t n_bits, int32_t width, uint16_t *X,
                        hipStream_t stream);

/*
 * Six feature classes of each scheme code (the code format of
 * patchwork_scheme_batch, Sec. 2): number of ovals clamped to 22; deepest
 * nesting clamped to 4; number of ovals at depth 1, 2, 3, 4 in the buckets
 * 0,1,2,3,4,5-6,7-9,10-14,15+.  labels is n x 6 int32.
 */
pw_status pw_features(const uint64_t *codes, int64_t n, int32_t *labels, hipStream_t stream);

/*
 * Softmax cross-entropy of the six heads of Y (n x 64 fp32; heads are the
 * column ranges [0,23) [23,28) [28,37) [37,46) [46,55) [55,64)) against
 * labels (n x 6), averaged over n: adds the loss to *loss and writes
 * dY = (softmax - onehot) / n as fp32 (dY32) and/or bf16 (dY16), each
 * may be NULL.
 */
pw_status pw_mlp_softmax_xent(const float *Y, const int32_t *labels, int64_t n, float *dY32, uint16_t *dY16,
                              float *loss, hipStream_t stream);

/*
 * out[j] = sum over rows k < n of X[k * cols + j] (bias gradients); with
 * accumulate != 0 the sums are added to out instead (out must then hold
 * valid values; the additions are atomic, in no fixed order).
 */
pw_status pw_mlp_colsum(const float *X, int64_t n, int32_t cols, float *out, int32_t accumulate,
                        hipStream_t stream);

/*
 * counts[start_h + labels[k * 6 + h]] += 1 over rows k < n and the six heads
 * (start_h = 0, 23, 28, 37, 46, 55; counts: 64 uint32, not zeroed here).
 * Labels must be valid classes of pw_features.
 */
pw_status pw_label_counts(const int32_t *labels, int64_t n, uint32_t *counts, hipStream_t stream);

/* x[i] = v for i < n. */
pw_status pw_fill_f32(float *x, int64_t n, float v, hipStream_t stream);

/*
 * Gradient of the novelty score (pw_mlp_score) of each row of Y with respect
 * to the logits, as bf16 (n x 64): for head h with p = softmax(Y_h) and
 * s_h = sum_j p_j rarity_j, d s_h / d Y_j = p_j (rarity_j - s_h).
 */
pw_status pw_mlp_score_grad(const float *Y, const float *rarity, int64_t n, uint16_t *dY16, hipStream_t stream);

/*
 * One Adam step (Kingma & Ba 2015, bias-corrected, step >= 1) on n fp32
 * weights w with gradient g and moments m, v; refreshes the bf16 copy w16
 * when it is not NULL.
 */
pw_status pw_mlp_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float beta1, float beta2,
                      float eps, int32_t step, uint16_t *w16, hipStream_t stream);

/* y[i] = x[i] rounded to bf16 (nearest even). */
pw_status pw_to_bf16(const float *x, int64_t n, uint16_t *y, hipStream_t stream);

/* out[c * rows + r] = in[r * cols + c]: the transpose of a rows x cols
 * bf16 matrix (the network keeps each weight matrix also as [out][in], so
 * that both operands of a forward product are contiguous along K).  in and
 * out must not overlap. */
pw_status pw_bf16_transpose(const uint16_t *in, int64_t rows, int64_t cols, uint16_t *out, hipStream_t stream);

/*
 * Novelty score of each row of Y (n x 64 logits): the sum over the six heads
 * of sum_j softmax(Y)_j * rarity[j] (rarity: 64 floats, e.g. -log of the
 * class frequencies seen so far).
 */
pw_status pw_mlp_score(const float *Y, const float *rarity, int64_t n, float *score, hipStream_t stream);

/*
 * Mutants: out[k] = parents[k mod n_parents] with `flips` bit positions in
 * [1, n_bits) toggled, each drawn from the SplitMix64 finaliser applied to a
 * key of (seed, k, flip index); bit 0 (sigma(0,0) = '+') is never touched.
 */
pw_status pw_mutate(const uint64_t *parents, int64_t n_parents, int64_t n, int32_t n_bits, int32_t flips,
                    uint64_t seed, uint64_t *out, hipStream_t stream);

/*
 * Flip distribution of each parent for guided mutation: cdf[p * 64 + j] =
 * P(flipped bit <= j) over bits 1 .. n_bits-1, where bit j has probability
 * (1 - explore) * softmax_j(gain / (temp * max |gain|)) + explore / (n_bits
 * - 1) and gain_j = -2 x_j dX[p * ldx + j] (x_j = +1 for '+', -1 for '-';
 * dX = gradient of the network's novelty score with respect to its input):
 * the first-order change of the score when bit j flips.  cdf: n_parents x
 * 64 floats; cdf[p*64] = 0, entries from n_bits - 1 on are 1.  n_bits <= 64.
 */
pw_status pw_flip_cdf(const uint64_t *parents, const float *dX, int64_t ldx, int64_t n_parents, int32_t n_bits,
                      float temp, float explore, float *cdf, hipStream_t stream);

/*
 * Guided mutants: out[k] = parents[p], p = k mod n_parents, with `flips` bits
 * toggled, each drawn from the parent's distribution in cdf (pw_flip_cdf)
 * by inverting a 24-bit uniform taken from the SplitMix64 finaliser applied
 * to a key of (seed, k, flip index).  Bit 0 is never drawn.
 */
pw_status pw_mutate_cdf(const uint64_t *parents, const float *cdf, int64_t n_parents, int64_t n, int32_t flips,
                        uint64_t seed, uint64_t *out, hipStream_t stream);

/*
 * Uniform masks: word w of mask k is the SplitMix64 output number
 * 2 (offset + k) + w of the stream seeded with `seed`; bits >= n_bits and
 * bit 0 cleared.
 */
pw_status pw_random_masks(uint64_t seed, uint64_t offset, int64_t n, int32_t n_bits, uint64_t *out,
                          hipStream_t stream);

/*
 * counts[b] += number of x[k] in [lo + b w, lo + (b+1) w), w = (hi - lo) /
 * bins; values outside [lo, hi) count in the end bins.  Used to find a
 * score threshold for the top fraction of candidates.
 */
pw_status pw_bin_floats(const float *x, int64_t n, float lo, float hi, int32_t bins, uint32_t *counts,
                        hipStream_t stream);

/*
 * Copies the candidates with score > threshold into out, in no particular
 * order, up to cap of them; *count (device, zeroed by the caller) receives
 * the number that passed, which may exceed cap.
 */
pw_status pw_select(const float *score, const uint64_t *cand, int64_t n, float threshold, uint64_t *out,
                    int64_t cap, unsigned long long *count, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PATCHWORK_H */
