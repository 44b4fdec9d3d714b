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
 * compile); idempotent.  Errors: PW_ERR_ARG (d > 9), PW_ERR_HIP (compile or
 * load failed; the handle keeps using the generic kernels).
 */
pw_status pw_tri_specialize(pw_tri_t tri);

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
 *   d_codes  n x 2 uint64 (lo, hi) written in input order.
 * n = 0 is a no-op; n < 0 is PW_ERR_ARG.
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
 * Many triangulations of uneven degree in one persistent launch (Sec. 3:
 * the second search mode sweeps many triangulations; kernel dispatch and
 * histogram aggregation are the costs at scale).
 *   tris      n_tris handles (host array), any mix of degrees.
 *   d_masks   one array of 128-bit masks (two uint64 per mask, whatever the
 *             degree); triangulation t owns masks [offsets[t], offsets[t+1]).
 *   offsets   host array of n_tris + 1 non-decreasing indices.
 *   hists     host array of n_tris histogram handles, or NULL; the witness
 *             of a code is its smallest global mask index.
 *   d_codes   NULL, or n x 2 uint64 codes written at the masks' positions.
 *   cfg       NULL for the defaults, or the tuned launch shape: masks per
 *             work item, waves per block (lowered until a block's LDS for
 *             the largest degree fits in 160 KiB), blocks per CU (0 = as
 *             many as the LDS allows).
 * Work items (chunks of one triangulation's masks) are taken from an atomic
 * queue in decreasing order of cost.  The call returns after the launch has
 * finished (its device tables are reused by the next call).
 */
typedef struct {
  int32_t chunk;
  int32_t waves_per_block;
  int32_t blocks_per_cu;
} pw_multi_config;

pw_status patchwork_scheme_batch_multi(const pw_tri_t *tris, int32_t n_tris, const void *d_masks,
                                       const int64_t *offsets, const pw_hist_t *hists, uint64_t *d_codes,
                                       const pw_multi_config *cfg, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PATCHWORK_H */
