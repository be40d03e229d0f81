/*
 * causal.h -- C ABI of the MI355X causal-set interval-abundance library (libcausal.so).
 *
 * The library computes, on one AMD Instinct MI355X (gfx950), the data-parallel path of
 * the causal-set action pipeline of W. J. Cunningham, "High Performance Algorithms for
 * Quantum Gravity and Cosmology" (2018):
 *
 *   cs_sprinkle            N points uniform in a spacetime region, labelled in time order
 *                          (App. A "Causal Set Sprinklings"; Sec. 3.2 "Pairwise Relations")
 *   cs_causal_matrix       the causal matrix as packed symmetric bitset rows P + P^T
 *                          (Sec. 3.2 "Data Structures for Graphs"; Ch. 4 introduction)
 *   cs_interval_histogram  interval abundances N_n (eq. IOIs; algorithms "Naive" and
 *                          "Optimized Interval Abundance Measurement"), two counters
 *   cs_action              Benincasa-Dowker action, local or smeared (Sec. 4.2)
 *   cs_dalembertian        discrete d'Alembertian of a scalar field (Sec. 4.1)
 *   cs_longest_chain       longest chains through Alexandroff sets (Sec. 2.5.2), and
 *   cs_degrees             the degree vectors of the matrix (Sec. 3.2)
 *   cs_batch_*             the four steps for an ensemble of independent 1+1 diamonds in
 *                          one persistent launch per step, capturable in a HIP graph
 *
 * Conventions for every entry point:
 *   - Pointers named "device" are caller-owned device memory (hipMalloc, or a torch CUDA
 *     tensor on ROCm).  The library never frees or retains caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Calls only
 *     validate arguments on the host and enqueue work; they return before it finishes.
 *   - Errors are returned synchronously as cs_status codes; argument errors enqueue
 *     nothing.  A launch failure reports CS_ERR_HIP; an earlier asynchronous fault is
 *     reported by whichever call observes it.  No C++ exception crosses the ABI.
 *   - Interval counts are exact integers: bit-exact results for the causal matrix and N_n.
 *   - n is limited to 2 <= n < 2^31 (CS_ERR_OVERFLOW above); memory bounds it earlier:
 *     the matrix takes n * cs_ld_words(n) * 8 bytes (2 GiB at n = 131072).
 */
#ifndef CAUSAL_H
#define CAUSAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CS_OK = 0,
    CS_ERR_INVALID_ARG = 1,  /* null pointer, n < 2, bad eps, ld too small ...        */
    CS_ERR_UNSUPPORTED = 2,  /* unknown region / counter / dimension                   */
    CS_ERR_WORKSPACE = 3,    /* workspace smaller than the matching *_workspace_bytes */
    CS_ERR_OVERFLOW = 4,     /* n >= 2^31, or a size that would overflow              */
    CS_ERR_HIP = 5,          /* a HIP runtime call or kernel launch failed            */
    CS_ERR_NO_DEVICE = 6     /* no gfx950 device is visible                           */
} cs_status;

/* Regions (App. A).  Coordinates are stored as SoA planes: coords[p * n + i].
 *   CS_MINK2_DIAMOND  1+1 Minkowski causal diamond in light-cone coordinates,
 *                     (u, v) uniform in [0,1)^2.  Planes: u, v.
 *                     i ≺ j  iff  u_i < u_j and v_i < v_j.
 *   CS_MINK4_DIAMOND  3+1 Minkowski Alexandrov interval of height 1 between (0,0) and
 *                     (1,0): uniform by rejection from [0,1) x [-1/2,1/2)^3.
 *                     Planes: t, x, y, z.  i ≺ j iff dt > 0 and dt^2 > (dx^2+dy^2)+dz^2.
 *   CS_DS4_SLAB       3+1 de Sitter slab, spherical foliation, conformal time
 *                     eta in [-eta0, eta0] with density ∝ sec^4(eta), uniform on S^3.
 *                     Planes: tan(eta), cos(eta), sin(eta), n0, n1, n2, n3 (unit vector).
 *                     i ≺ j iff eta_i < eta_j and cos(eta_j - eta_i) < n_i . n_j.
 *   CS_DS2_SLAB       1+1 de Sitter slab, spherical foliation (Sec. 4.3, the benchmark
 *                     of the action): metric sec^2(eta)(-d eta^2 + d theta^2), eta in
 *                     [-eta0, eta0] with density ∝ sec^2(eta), theta uniform on [0, 2 pi).
 *                     tan(eta) is uniform: x = (2u - 1) tan(eta0), eta = atan(x),
 *                     theta = 2 pi w.  Planes: x = tan(eta), eta, theta.
 *                     i ≺ j iff eta_i < eta_j and pi - |pi - |theta_i - theta_j|| <
 *                     eta_j - eta_i (the angle measured the short way round).
 *   CS_MINK3_DIAMOND  2+1 Minkowski Alexandrov interval of height 1: uniform by rejection
 *                     from [0,1) x [-1/2,1/2)^2.  Planes: t, x, y.
 *                     i ≺ j iff dt > 0 and dt^2 > dx^2 + dy^2.
 * Relations are strict: null-separated and equal-time pairs are unrelated.  All
 * predicates are evaluated in IEEE fp64 in the order written, without contraction. */
enum { CS_MINK2_DIAMOND = 0, CS_MINK4_DIAMOND = 1, CS_DS4_SLAB = 2, CS_DS2_SLAB = 3,
       CS_MINK3_DIAMOND = 4 };

/* Interval counters (all four give identical, exact results). */
enum {
    CS_COUNT_BITSET = 0,   /* VALU: 32-bit AND + popcount over LDS-staged row words, on
                              the related pairs only (Alg. "Optimized Interval Abundance
                              Measurement"): a 128 x 128 tile's related pairs are packed
                              into tasks of one row and up to four related columns; tiles
                              where more than about half the pairs are related take the
                              dense product of CS_COUNT_BITSET_DENSE instead              */
    CS_COUNT_MFMA = 1,     /* dense C.C on int8 MFMA (v_mfma_i32_32x32x32_i8), int32 acc  */
    CS_COUNT_MFMA_FP4 = 2, /* dense C.C on fp4 MFMA (v_mfma_scale_f32_32x32x64_f8f6f4,
                              e2m1 operands 0 / 1.0, unit scales), f32 acc started at 2^23:
                              exact because every product is 0 or 1 and 2^23 + count stays
                              below 2^24; needs n <= 2^23 + 1 for the histogram (n < 2^24
                              for the d'Alembertian), CS_ERR_OVERFLOW otherwise           */
    CS_COUNT_BITSET_DENSE = 3  /* VALU AND + popcount over every pair of each tile that
                              holds a related pair (8 x 8 pairs per thread), unrelated
                              pairs discarded at binning: the dense reference of the
                              related-pair counter                                        */
};

/* Number of fp64 coordinate planes of a region (2, 4, 7, 3 or 3); -1 if unknown. */
int cs_coord_planes(int region);

/* Row stride of the packed matrix in uint64 words: n rounded up to 512 bits. */
int64_t cs_ld_words(int64_t n);

/* Human-readable name of a status code (static string). */
const char *cs_status_string(cs_status s);

/* Device workspace needed by cs_sprinkle for (region, n), in bytes. */
size_t cs_sprinkle_workspace_bytes(int region, int64_t n);

/*
 * Sprinkle n points into `region` from `seed` and store them time-ordered.
 *   eta0       half-width of the de Sitter slab in conformal time, 0 < eta0 < pi/2
 *              (ignored for the Minkowski diamonds).
 *   seed       64-bit seed of the counter-based generator (SplitMix64 outputs).
 *   coords     device, cs_coord_planes(region) * n doubles, written as SoA planes.
 *   workspace  device, at least cs_sprinkle_workspace_bytes(region, n) bytes.
 * Order: 1+1 by the exact integer (u + v) * 2^53, 3+1 diamond by t, de Sitter by
 * tan(eta); ties by generation index.  Every relation then has i < j.
 * The 3+1 diamond keeps the first n accepted candidates in candidate order.
 */
cs_status cs_sprinkle(int region, double eta0, uint64_t seed, int64_t n, double *coords,
                      void *workspace, size_t workspace_bytes, void *stream);

/*
 * Causal matrix S = C + C^T of n time-ordered points (C strictly upper triangular).
 *   coords  device, SoA planes as written by cs_sprinkle.  The points must be labelled
 *           in time order, as cs_sprinkle writes them (non-decreasing time plane; in the
 *           1+1 diamond any linear extension of the order): only pairs i < j are tested,
 *           and in the 2+1 and 3+1 diamonds the test takes t_j >= t_i as given.
 *   bits    device, n * ld_words uint64.  Bit j of row i is bit (j & 63) of word
 *           bits[i * ld_words + (j >> 6)].  Every word is written, padding bits as 0.
 *   ld_words >= cs_ld_words(n) (CS_ERR_INVALID_ARG otherwise).
 */
cs_status cs_causal_matrix(int region, const double *coords, int64_t n, uint64_t *bits,
                           int64_t ld_words, void *stream);

/* Device workspace needed by cs_interval_histogram, in bytes. */
size_t cs_histogram_workspace_bytes(int64_t n, int counter);

/*
 * Interval abundances: hist[m] = N_m = number of pairs i < j with i ≺ j and exactly m
 * elements k with i ≺ k ≺ j, for m = 0 .. n-2 (the thesis's n_{m+1}).
 *   bits     device, the matrix from cs_causal_matrix (n rows, ld_words stride).
 *   counter  CS_COUNT_BITSET, CS_COUNT_MFMA, CS_COUNT_MFMA_FP4 or CS_COUNT_BITSET_DENSE;
 *            identical results.
 *   hist     device, n-1 uint64, overwritten (zeroed by the callee).
 *   workspace device, at least cs_histogram_workspace_bytes(n, counter) bytes.
 * The MFMA counters address a 256-row panel of the matrix with 32-bit offsets and
 * need ld_words <= 2^19 (a panel below 1 GiB, n up to 33.5 million); larger strides
 * give CS_ERR_OVERFLOW.  CS_COUNT_MFMA_FP4 also needs n <= 2^23 + 1.
 */
cs_status cs_interval_histogram(const uint64_t *bits, int64_t n, int64_t ld_words, int counter,
                                uint64_t *hist, void *workspace, size_t workspace_bytes,
                                void *stream);

/*
 * cs_interval_histogram without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, limits and results as cs_interval_histogram; the counters'
 * scratch memory is a static device array of the library (16 KiB, one copy per GPU, held
 * until the process ends), so this call allocates nothing.  A counter whose workspace
 * (cs_histogram_workspace_bytes) exceeds that array gives CS_ERR_WORKSPACE.  Every call on
 * one GPU shares the array: calls on one GPU that overlap in time (on different streams,
 * or from host threads without ordering) race and must be serialised by the caller.
 */
cs_status cs_interval_histogram_noalloc(const uint64_t *bits, int64_t n, int64_t ld_words,
                                        int counter, uint64_t *hist, void *stream);

/* Device workspace needed by cs_dalembertian, in bytes (0 for a bad n or counter). */
size_t cs_dalembertian_workspace_bytes(int64_t n, int counter);

/*
 * Discrete d'Alembertian of a scalar field on the causal set (Sec. 4.1, eqs. b2d_local and
 * b4d_local), for every element j:
 *   B phi(j) = (K / ell^2) [ -phi(j) + sum_m c_m sum_{i in L_m(j)} phi(i) ],
 *   L_m(j) = { i ≺ j with exactly m-1 elements strictly between i and j },
 *   dim = 2: K = 2,          (c_1, c_2, c_3)      = (2, -4, 2)
 *   dim = 3: K = C_3,        (c_1, c_2, c_3)      = (1, -27/8, 9/4)      (eq. b3d_local)
 *   dim = 4: K = 4/sqrt(6),  (c_1, c_2, c_3, c_4) = (1, -9, 16, -8),
 * with C_3 = (pi / (3 sqrt 2))^(2/3) / Gamma(5/3).
 *   bits     device, the matrix from cs_causal_matrix (n rows, ld_words stride).
 *   ell      discreteness scale (> 0), nu^(-1/(d+1)) for sprinkling density nu.
 *   counter  CS_COUNT_MFMA or CS_COUNT_MFMA_FP4 (the interval sizes come from the same
 *            tiles as cs_interval_histogram; the bitset counter gives CS_ERR_UNSUPPORTED).
 *   phi      device, n doubles (time-ordered like the points).
 *   out      device, n doubles, overwritten.
 *   workspace device, at least cs_dalembertian_workspace_bytes(n, counter) bytes.
 * The sums over L_m(j) are accumulated in fp64 by atomic adds in an order that varies
 * between runs, so each out[j] is exact up to the rounding of a sum of its summands.
 * Same limits as cs_interval_histogram for the MFMA counters.
 */
cs_status cs_dalembertian(const uint64_t *bits, int64_t n, int64_t ld_words, int dim, double ell,
                          int counter, const double *phi, double *out, void *workspace,
                          size_t workspace_bytes, void *stream);

/* Device workspace needed by cs_longest_chain, in bytes (0 for a bad n or count):
 * about 17 * n * count bytes, plus 4n. */
size_t cs_longest_chain_workspace_bytes(int64_t n, int64_t count);

/*
 * Longest chains through Alexandroff sets (Sec. 2.5.2 "Set Partitions", algorithm
 * "Maximal Chain Length"), for `count` pairs at once.  Index -1 names a virtual element
 * below every element and index n one above every element; a chain's length is its
 * number of links.  For pair s:
 *   length[s]          links on the longest chain from lo[s] to hi[s] through
 *                      A = {k : lo[s] ≺ k ≺ hi[s]}; 0 when lo[s] does not precede hi[s].
 *                      For (lo, hi) = (-1, n) this is the height of the whole order + 1.
 *   height[s*n + k]    when height is not NULL: links on the longest chain from lo[s] to k,
 *                      for k in A or k = hi[s] (when lo[s] ≺ hi[s]); 0 for every other k.
 *                      With lo[s] = -1 this is one more than the longest distance from a
 *                      minimal element to k (the antichain partition of the boundary
 *                      algorithms, Sec. 5.4).
 *   bits       device, the matrix from cs_causal_matrix (n rows, ld_words stride): labels
 *              must be a linear extension of the order (i ≺ j implies i < j), as
 *              cs_sprinkle + cs_causal_matrix produce them.
 *   lo, hi     HOST arrays of count int64: -1 <= lo[s] < hi[s] <= n, lo[s] < n, hi[s] >= 0
 *              (CS_ERR_INVALID_ARG otherwise).  1 <= count <= 65535 (CS_ERR_OVERFLOW above).
 *   length     device, count int32, overwritten.
 *   height     device, count * n int32, overwritten; or NULL.
 *   workspace  device, at least cs_longest_chain_workspace_bytes(n, count) bytes.
 * Unlike the other calls this one returns only after the work is done: it removes the
 * minimal elements of each set round by round (one round per link of the longest chain)
 * and reads a progress count back from the device between batches of rounds, which
 * synchronizes `stream`.  Results are exact integers.
 */
cs_status cs_longest_chain(const uint64_t *bits, int64_t n, int64_t ld_words, const int64_t *lo,
                           const int64_t *hi, int64_t count, int32_t *length, int32_t *height,
                           void *workspace, size_t workspace_bytes, void *stream);

/*
 * Degree vectors (Sec. 3.2): for every element k, indeg[k] = number of elements
 * preceding k and outdeg[k] = number of elements k precedes (with time-ordered labels:
 * the set bits of row k below and above column k).  Minimal elements have indeg 0,
 * maximal ones outdeg 0.
 *   bits    device, the matrix from cs_causal_matrix.
 *   indeg, outdeg  device, n int64 each, overwritten; either may be NULL, not both.
 */
cs_status cs_degrees(const uint64_t *bits, int64_t n, int64_t ld_words, int64_t *indeg,
                     int64_t *outdeg, void *stream);

/*
 * Benincasa-Dowker action from the abundances (l = l_p).
 *   dim = 2: eps == 0: S = 2 (N - 2N_0 + 4N_1 - 2N_2)
 *            eps > 0 : S = 2 eps [N - 2 eps sum_m N_m f_2(m, eps)]
 *   dim = 3: eps == 0: S = C_3 (N - N_0 + (27/8) N_1 - (9/4) N_2)
 *            eps > 0 : S = C_3 eps^(2/3) [N - eps sum_m N_m f_3(m, eps)]
 *            with C_3 = (pi / (3 sqrt 2))^(2/3) / Gamma(5/3) (eqs. s3d_local, f_3)
 *   dim = 4: eps == 0: S = (4/sqrt 6)(N - N_0 + 9N_1 - 16N_2 + 8N_3)
 *            eps > 0 : S = 4 sqrt(eps/6) [N - eps sum_m N_m f_4(m, eps)]
 *   0 <= eps <= 1; at eps = 1 the smeared form equals the local one.
 *   hist  device, n-1 uint64.   out  device, one double.
 * The local combination is an exact int64; the smeared sum is accumulated in
 * double-double (weights included), then rounded once to fp64.  Bins past the point
 * where (1 - eps)^m < e^-700 are not visited: all their terms together are below 2^-820.
 */
cs_status cs_action(const uint64_t *hist, int64_t n, int dim, double eps, double *out,
                    void *stream);

/* ---------------------------------------------------------------------------------
 * Ensembles: `count` independent 1+1 diamonds of sizes n[k] (2 <= n[k] <= 8192).
 * cs_batch_plan builds a plan (sizes, offsets, work lists, tile choice); its work
 * tables are uploaded once to device memory that the plan owns (freed by cs_batch_free).
 * cs_batch_run enqueues the whole pipeline -- sprinkle, matrix, counts, actions --
 * as a fixed sequence of kernels with no host synchronisation and no allocation, so
 * the caller may capture it in a HIP graph.
 *   seeds      device, count uint64.
 *   workspace  device, cs_batch_workspace_bytes(plan) bytes.
 *   hist       device, cs_batch_hist_len(plan) uint64: instance k's N_m at
 *              hist[cs_batch_hist_offset(plan, k) + m], m = 0 .. n[k]-2.
 *   actions    device, count * n_eps doubles: actions[k * n_eps + e] for eps[e]
 *              (eps[e] == 0 selects the local action).
 * --------------------------------------------------------------------------------- */
typedef struct cs_batch_plan_t *cs_batch_plan_handle;

cs_status cs_batch_plan(int64_t count, const int64_t *n /* host */, int counter,
                        int n_eps, const double *eps /* host */, const char *tune_cache,
                        cs_batch_plan_handle *plan);
size_t cs_batch_workspace_bytes(cs_batch_plan_handle plan);
int64_t cs_batch_hist_len(cs_batch_plan_handle plan);
int64_t cs_batch_hist_offset(cs_batch_plan_handle plan, int64_t k);
/*
 * Where a run leaves instance k's intermediate results in the caller's workspace: byte
 * offsets of its time-ordered coordinates (u then v, n[k] doubles each, as
 * cs_sprinkle writes them) and of its packed matrix (n[k] rows of cs_ld_words(n[k])
 * uint64 words, as cs_causal_matrix writes it).  -1 for a null plan or k out of range.
 * The contents are valid after a run until the workspace is reused.
 */
int64_t cs_batch_coords_offset(cs_batch_plan_handle plan, int64_t k);
int64_t cs_batch_bits_offset(cs_batch_plan_handle plan, int64_t k);
cs_status cs_batch_run(cs_batch_plan_handle plan, const uint64_t *seeds, uint64_t *hist,
                       double *actions, void *workspace, size_t workspace_bytes, void *stream);
cs_status cs_batch_free(cs_batch_plan_handle plan);

/*
 * HIP graph of one cs_batch_run with these buffers, captured on an internal stream and
 * instantiated (so the graph replays the same four launches: sprinkle, which also clears
 * the histograms and the work counters, build, count, action).  graph_exec receives an opaque hipGraphExec_t owned by the caller:
 * launch it with cs_batch_graph_launch on any stream, release it with
 * cs_batch_graph_destroy.  The buffers must stay valid while the graph is in use.
 */
cs_status cs_batch_graph_create(cs_batch_plan_handle plan, const uint64_t *seeds, uint64_t *hist,
                                double *actions, void *workspace, size_t workspace_bytes,
                                void **graph_exec);
cs_status cs_batch_graph_launch(void *graph_exec, void *stream);
cs_status cs_batch_graph_destroy(void *graph_exec);

/*
 * Tile autotuner (project-written) of the ensemble counters.  Instance sizes fall in four
 * buckets, [2, 1023], [1024, 2047], [2048, 4095] and [4096, 8192].  For each requested
 * counter and bucket it times, on the current device, every tile configuration of the
 * counter on an ensemble of diamonds with sizes spread evenly around the bucket's centre
 * (768, 1536, 3072 or 6144 points, from 2c - hi to hi; enough of them that their row
 * panels of 128-row tiles number sixteen per compute unit, at least 16; the counting
 * launches only, best of five, HIP events on `stream`):
 *   CS_COUNT_MFMA, CS_COUNT_MFMA_FP4: 128x128 output tiles with two or with one
 *       persistent workgroup per compute unit, 256x256 tiles with one;
 *   CS_COUNT_BITSET: related-pair tiles with at most 2304 or 1152 tasks (denser tiles
 *       take the dense product), two workgroups per CU; the same with one; and the dense
 *       product on every tile.
 *   n_bucket   0: every bucket; else the bucket holding this size (2 .. 8192).
 *   counter    CS_COUNT_BITSET, CS_COUNT_MFMA, CS_COUNT_MFMA_FP4, or -1 for all three.
 * The fastest configuration of each (counter, bucket) is stored in the JSON file
 * cache_path (one entry per line, keeping the entries of an existing file that were not
 * re-tuned).  cs_batch_plan reads its own counter's entries from `tune_cache` (may be
 * NULL); without an entry it uses 128 tiles with two workgroups per CU (MFMA) and
 * related-pair tiles with at most 2304 tasks (bitset).  The tuner allocates and
 * frees its own device memory and synchronises `stream`.  Every configuration gives
 * identical, exact histograms.
 */
cs_status cs_autotune(const char *cache_path, int64_t n_bucket, int counter, void *stream);

/*
 * Measurement utility (not part of the pipeline): the int8 (counter = CS_COUNT_MFMA) or fp4
 * (CS_COUNT_MFMA_FP4) MFMA throughput this device sustains, in TOP/s, from a register-only
 * MFMA stream on every CU (best of two timed launches after a warm-up).  Allocates and frees
 * a few KiB of device memory and synchronises `stream`.  *tops is host memory.
 */
cs_status cs_measure_mfma_peak(int counter, double *tops, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CAUSAL_H */
