/*
 * zeta3.h -- C ABI of libzeta3, the MI355X (gfx950) harmonic-basis 3PCF estimator.
 *
 * The library computes the binned multipole estimator of the three-point correlation
 * function of a spin-0 field on the sphere (arXiv 2408.16847, section "3PCF binned
 * estimator", eqs. Xm.binned, Ym/Zm.binned, zetamEst, zetamEst2; resummation eq.
 * eq_zeta_harmonic):
 *
 *   a_{m,b}(p)    = sum_{j in bin b of p} w_j x_j exp(-i m phi_pj)       (multipoles)
 *   W_{p,b}       = sum_{j in bin b of p} w_j
 *   X_m(b; p)     = a_{m,b}(p) / W_{p,b}     (0 when W_{p,b} = 0)          (normalise)
 *   zeta_m(b1,b2) = (1 / sum_p w_p) sum_p w_p x_p X_m(b1; p) conj(X_m(b2; p))  (contract)
 *   zeta(b1,b2,phi) = sum_{|m|<=M} zeta_m exp(i m phi),  zeta_{-m} = conj(zeta_m)
 *
 * phi_pj is the position angle of neighbour j seen from pivot p, measured from local
 * north through east.  A neighbour j is in bin b of pivot p iff
 * E_b <= d2 < E_{b+1} where d2 = (dx*dx + dy*dy) + dz*dz is the squared chord
 * computed in FP64 with each operation rounded separately, dx = x_j - x_p, and
 * E_0 < ... < E_nbins is the caller's chord-squared edge table (E = (2 sin(theta/2))^2).
 * A pivot is never its own neighbour because E_0 > 0 is required.
 *
 * Conventions common to every entry point
 * ---------------------------------------
 *  - Array arguments are DEVICE pointers owned by the caller unless marked [host].
 *  - "stream" is a hipStream_t passed as void* (NULL = the legacy default stream).
 *    Every call only enqueues work on that stream and returns; the exceptions are
 *    z3_build_index (synchronises on the stream to size its tables) and z3_sync.
 *  - Every function returns a z3_status and never throws.  On Z3_ERR_INVALID_ARG no
 *    output has been written.  The text of the last error of the calling thread is
 *    returned by z3_last_error().  Asynchronous device faults surface as Z3_ERR_HIP
 *    from the next call or from z3_sync.
 *  - zeta arrays are FP64 [m_max+1][nbins][nbins][2] (re, im), full Hermitian matrices,
 *    and are ACCUMULATED (+=), so pivot ranges can be processed in pieces and summed.
 *  - Pivots are the catalogue's own points, addressed by their position in the index
 *    order (see z3_index_perm), so that pivot ranges [p0, p1) can be streamed; only
 *    z3_estimate_pivots takes an external pivot catalogue.
 */
#ifndef ZETA3_H
#define ZETA3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct z3_index_s *z3_index;

typedef enum {
    Z3_OK = 0,
    Z3_ERR_INVALID_ARG = 1,   /* bad sizes, NULL pointers, unsorted edges, ...         */
    Z3_ERR_OUT_OF_MEMORY = 2, /* device allocation failed                               */
    Z3_ERR_HIP = 3,           /* a HIP runtime call or a kernel failed                  */
    Z3_ERR_UNSUPPORTED = 4,   /* valid request outside what this library implements     */
    Z3_ERR_OVERFLOW = 5       /* catalogue or pair count beyond the supported range     */
} z3_status;

enum {
    Z3_PREC_FP64 = 0,  /* all arithmetic in FP64                                         */
    Z3_PREC_MIXED = 1  /* multipoles formed in FP64 (separations, bins, bearing,
                          harmonics, sums) and stored in FP32; split-FP32 MFMA contraction
                          with FP64 sums; many-map kernel: FP64 harmonics rounded once,
                          FP32 MFMA products added into FP64 */
};

enum {
    Z3_NORM_BIN = 0,  /* X = a / W_{p,b} (the per-bin average of the estimator)          */
    Z3_NORM_NONE = 1  /* raw sums a_{m,b}; callers can apply any other normaliser       */
};

enum {
    /* z3_estimate_ex: leave out the triangles whose two neighbours are the same point
       (k = j), which the product X_m(b) conj X_m(b) of eq. zetamEst otherwise holds on the
       diagonal b1 = b2 (the overcount noted in the kappa^3 multipole-signal subsection) */
    Z3_EST_EXCLUDE_SELF = 1u << 0
};

/* Largest supported multipole and bin count. */
#define Z3_MAX_MMAX 16
#define Z3_MAX_NBINS 64
/* Angular-histogram estimator: bins per circle and largest multipole (m_max < n_phi / 2). */
#define Z3_MAX_NPHI 256
#define Z3_MAX_MMAX_HIST 127

/*
 * Build the sky-cell index of a catalogue of n points (the neighbour search of the
 * binned estimator; it replaces the paper's tree search with a latitude-band x
 * longitude-cell grid, points sorted by cell).
 *   n              number of points, 0 <= n < 2^29 (Z3_ERR_OVERFLOW above)
 *   xyz            [3][n] FP64 unit vectors (x row, y row, z row); | |r|^2 - 1 | above
 *                  1e-10 for any point, or a non-finite coordinate, is Z3_ERR_INVALID_ARG
 *   w              [n] FP64 weights w_i (eq. of the discrete field), or NULL for all 1
 *   nbins          1 .. Z3_MAX_NBINS
 *   edges_chord2   [host] nbins+1 strictly increasing chord-squared edges, 0 < E_0,
 *                  E_nbins <= 4
 *   cell_size      band height in radians; <= 0 selects 1.4 * sqrt(A / n) where A is
 *                  the area of the catalogue's colatitude range (about two HEALPix rings)
 *   out            receives the index; free it with z3_index_free
 * Synchronises on `stream` (to size its tables, and before it returns).  The input arrays
 * may be freed after it returns.
 */
z3_status z3_build_index(int64_t n, const double *xyz, const double *w, int nbins,
                         const double *edges_chord2, double cell_size, void *stream,
                         z3_index *out);

/*
 * Attach field values: nmaps maps of n values each, x [nmaps][n] FP64 in the
 * catalogue's original order.  The index stores w_i x_i in index order and, per map,
 * 32-byte neighbour records {x, y, z, w x} (2 n records: every latitude band is stored
 * twice in a row).  Waits for earlier work on `stream`; replaces values attached before.
 */
z3_status z3_index_set_values(z3_index idx, int nmaps, const double *x, void *stream);

/*
 * Replace the values of the attached maps in place: x [nmaps][n] FP64 (catalogue order),
 * nmaps as attached by z3_index_set_values.  Enqueues kernels only on `stream` (no host
 * synchronisation, no allocation), so it can be captured in a HIP graph with the estimator
 * and the adjoint; work already queued on other streams that reads the old values must be
 * ordered before it by the caller.  Tuned block shapes are kept.
 */
z3_status z3_index_update_values(z3_index idx, const double *x, void *stream);

/*
 * Graph capture.  The estimator and adjoint calls take their chunk workspaces from the
 * library's stream-ordered memory pool and keep them per device for later calls (held until
 * the process ends; a call that needs more than every idle block gives those back first; a
 * call waits for a kept block's last use, on whatever stream, before it uses the block);
 * while their stream is being captured into a HIP
 * graph they take them instead from a workspace held by the index, so that the captured
 * kernels point at memory that stays valid for every replay.  This call reserves that
 * workspace: max(min_bytes, the largest total any eager call on this index has used so
 * far) bytes, kept until z3_index_free; [host] reserved (may be NULL) receives the size.
 * Run each call once eagerly with the arguments it will be captured with, then prepare,
 * then capture.  A captured call whose needs exceed the reservation fails with
 * Z3_ERR_INVALID_ARG (and the capture is then unusable).  Synchronises the device.  Growing
 * the reservation allocates a new workspace for later captures and keeps the previous one
 * (graphs captured before still point at it) until z3_index_free.  Graphs captured on one
 * index may share a workspace: their replays must not overlap in time.
 * z3_contract and z3_build_index / z3_index_set_values cannot be captured, nor should
 * z3_estimate_pivots and z3_estimate_cross_catalogues be: their pivot sort is rocPRIM's
 * radix sort, whose launches are not part of what the library checks under capture.
 */
z3_status z3_index_prepare_capture(z3_index idx, size_t min_bytes, size_t *reserved);

/* Sizes of an index ([host] outputs, any may be NULL). */
z3_status z3_index_info(z3_index idx, int64_t *n, int *nbins, int *nmaps, int *nbands,
                        int64_t *ncells);

/* perm [n] int64: original catalogue index of the point at index position i. */
z3_status z3_index_perm(z3_index idx, int64_t *perm, void *stream);

/*
 * Block shape of the MFMA many-map kernel (z3_estimate_maps with more than 56 maps on the
 * FP64 path or 24 on the mixed path, z3_adjoint_maps with more than 56): one block per
 * pivot with `waves` wave64s, each owning `maps_per_wave` maps; compiled shapes are (4, 16),
 * (2, 32), (2, 16) and (4, 32).  A fixed shape also selects the MFMA kernel for any count
 * above 4 maps.  (0, 0), the default, lets the library time every compiled shape on a
 * 4096-pivot sample of the first eager call for each (m_max, prec) and keep the fastest for
 * this index.  Every shape gives bit-identical results.  Attaching new values
 * (z3_index_set_values) forgets the tuned shapes.  Z3_ERR_INVALID_ARG for a shape that is
 * not compiled.
 */
z3_status z3_index_set_batch_shape(z3_index idx, int waves, int maps_per_wave);

/* [host] The fixed or tuned shape for (m_max, prec); (0, 0) if not tuned yet. */
z3_status z3_index_batch_shape(z3_index idx, int m_max, int prec, int *waves, int *maps_per_wave);

/*
 * Index of a catalogue on a plane (the estimator is the same for pivots on any smooth
 * manifold; the paper's code offers the sphere and the plane, see its description of the
 * cBalls code):
 *   xy        [2][n] FP64 positions (x row, y row), any units, finite
 *   w         [n] weights or NULL
 *   edges_d2  [host] nbins+1 strictly increasing squared distances, 0 < E_0
 *   cell_size strip height in the units of xy; <= 0 selects 1.4 x the mean spacing
 * Pairs: d2 = dx*dx + dy*dy in FP64, E_b <= d2 < E_{b+1}; the angle of a separation is
 * measured from the +y axis towards +x.  The index serves z3_index_set_values,
 * z3_accumulate_multipoles, z3_estimate, z3_estimate_ex, z3_estimate_cross, z3_adjoint,
 * z3_estimate_maps and z3_adjoint_maps (one-map passes per map), z3_estimate_pivots and
 * z3_estimate_cross_catalogues, whose pivot positions are then [2][npiv] (x row, y row).
 * Synchronises on `stream`.
 */
z3_status z3_build_index_planar(int64_t n, const double *xy, const double *w, int nbins,
                                const double *edges_d2, double cell_size, void *stream,
                                z3_index *out);

/* Release an index and its device memory (NULL is ignored).  Waits for its work. */
void z3_index_free(z3_index idx);

/*
 * Per-pivot multipoles (eqs. Xm.binned, Ym/Zm.binned) for pivots [p0, p1) in index
 * order, map `map` of the attached values.  P = p1 - p0.
 *   A       [m_max+1][2][nbins][P]: re and im of X_m(b; p) (or raw a with Z3_NORM_NONE);
 *           FP64 for Z3_PREC_FP64, FP32 for Z3_PREC_MIXED.  May be NULL.
 *   W       [nbins][P] FP64 W_{p,b}, or NULL
 *   counts  [nbins][P] int64 N_{p,b}, or NULL
 *   idhash  [nbins][P] uint64: sum over the bin's neighbours j of SplitMix64(j), j the
 *           original catalogue index (an order-independent fingerprint of the
 *           neighbour list), or NULL
 *   pair_total [1] uint64, += the number of pairs found, or NULL
 */
z3_status z3_accumulate_multipoles(z3_index idx, int map, int m_max, int prec, int norm,
                                   int64_t p0, int64_t p1, void *A, double *W,
                                   int64_t *counts, uint64_t *idhash, uint64_t *pair_total,
                                   void *stream);

/*
 * Contraction (eq. zetamEst / zetamEst2) of materialised multipoles:
 *   zeta[m][b1][b2] += sum_p v_p X_m(b1; p) conj(X_m(b2; p))
 * A has the layout written by z3_accumulate_multipoles (FP64 or FP32 per prec);
 * piv_v [npiv] FP64 pivot products w_p x_p.  Not divided by sum_p w_p (z3_finalize).
 */
z3_status z3_contract(int64_t npiv, int m_max, int nbins, int prec, const void *A,
                      const double *piv_v, double *zeta, void *stream);

/*
 * Fused estimator for pivots [p0, p1) of map `map`: multipoles per pivot chunk into a
 * library-owned workspace, then the contraction, zeta += (unnormalised), and
 * pair_total += pairs (may be NULL).  Equivalent to accumulate + contract.
 */
z3_status z3_estimate(z3_index idx, int map, int m_max, int prec, int64_t p0, int64_t p1,
                      double *zeta, uint64_t *pair_total, void *stream);

/*
 * z3_estimate with options.  flags: 0 or Z3_EST_EXCLUDE_SELF (other bits:
 * Z3_ERR_INVALID_ARG).  With Z3_EST_EXCLUDE_SELF the k = j terms are removed:
 *   zeta_m[b][b] re -= sum_p w_p x_p Q_{p,b} / W_{p,b}^2,  Q_{p,b} = sum_{j in b} (w_j x_j)^2
 * for every m (0 where W_{p,b} = 0), accumulated in FP64 on either precision path, so that
 * zeta holds the triplet sum over k != j; the other entries are those of z3_estimate.
 * Same arguments, chunking and accumulation (zeta +=, unnormalised) as z3_estimate;
 * the removal adds a workspace of 8 x nbins bytes per 64 pivots of a chunk.  With the flag
 * Z3_PREC_MIXED stores and contracts the multipoles in FP64 (as Z3_PREC_FP64 does): the
 * removed self terms can be most of |X_m(b)|^2, and FP32 storage would leave an error
 * relative to the full product rather than to the smaller result.
 */
z3_status z3_estimate_ex(z3_index idx, int map, int m_max, int prec, unsigned flags, int64_t p0,
                         int64_t p1, double *zeta, uint64_t *pair_total, void *stream);

/*
 * The fused estimator of z3_estimate_ex (same arguments, same results up to the order of
 * the FP64 chunk sums) for callers that cannot allocate device memory: code being captured
 * into a HIP graph, tight serving loops, harnesses that forbid allocation.  It calls no
 * hipMalloc, hipFree or other allocating routine and records no timing events; its chunk
 * workspace is a static 512 MiB device array built into the library (one per GPU, held
 * from the first call on that GPU until the process ends), which also bounds the pivot
 * chunk: about 150,000 pivots per chunk in FP64 and 300,000 on the mixed path at
 * 20 bins and m_max = 10.  Z3_ERR_UNSUPPORTED if one block of 256 pivots does not fit
 * (not reached within Z3_MAX_MMAX and Z3_MAX_NBINS).  Every call on a GPU shares that
 * GPU's array and leaves its last contents there; calls that overlap on one GPU (several
 * streams or threads) race and must be serialised by the caller.
 */
z3_status z3_estimate_static(z3_index idx, int map, int m_max, int prec, unsigned flags, int64_t p0,
                             int64_t p1, double *zeta, uint64_t *pair_total, void *stream);

/*
 * Angular bins of the histogram estimator (the complexity discussion of the "3PCF binned
 * estimator" subsection: histograms around each pivot in radial and n_phi angular bins,
 * then a Fourier transform over the angular bins).  bounds [host] [n_phi][2] FP64 holds the
 * boundary directions (cos, sin)(2 pi k / n_phi), k = 0..n_phi-1 (angular bin k covers the
 * bearings [2 pi k, 2 pi (k+1)) / n_phi, measured from local north towards east); every
 * row must lie within 1e-15 of those values (Z3_ERR_INVALID_ARG otherwise), 4 <= n_phi <=
 * Z3_MAX_NPHI.  The pair's bin is decided by sign tests against exactly these numbers:
 * bin k iff c_k u2 - s_k u1 >= 0 and c_{k+1} u2 - s_{k+1} u1 < 0, with (u1, u2) the
 * separation's components on the unnormalised local north N = (-z x, -z y, 1 - z z)
 * (N = (1 - x x, -x y, -x z) where (N.N) < 1e-24) and east E = N x r_p, every product and
 * sum rounded on its own and summed as (x + y) + z.  Sky indexes only (Z3_ERR_UNSUPPORTED
 * on a plane).  Allocates and copies synchronously; replaces earlier bins of the index.
 */
z3_status z3_index_set_phi_bins(z3_index idx, int n_phi, const double *bounds);

/*
 * Per-pivot multipoles of the histogram estimator for pivots [p0, p1) in index order:
 *   H_{p,b,k} = sum of w_j x_j over the pairs of radial bin b and angular bin k,
 *   a_{m,b}(p) = sum_k H_{p,b,k} exp(-i m (k + 1/2) dphi)   (each pair at its bin centre),
 * then X = a / W_{p,b} (Z3_NORM_BIN) as in z3_accumulate_multipoles, for
 * 0 <= m_max < n_phi / 2 (and <= Z3_MAX_MMAX_HIST).  Outputs as z3_accumulate_multipoles
 * (A [m_max+1][2][nbins][P] FP64 or FP32 per prec, W, counts; each may be NULL), plus
 *   counts_phi [nbins][n_phi][P] int32 pairs per (pivot, radial bin, angular bin), or NULL
 * (LDS per block of 256 threads: 32 n_phi (64/L + 1) bytes, 48 n_phi (64/L + 1) with
 * counts_phi, plus 48 n_phi, where L, the lanes per pivot, is the least power of two up to 16
 * with n_phi <= 18 L: at most 74 KB; Z3_ERR_UNSUPPORTED beyond the device's limit).  Sums are FP64 on both precisions.
 */
z3_status z3_accumulate_histogram(z3_index idx, int map, int m_max, int prec, int norm, int64_t p0,
                                  int64_t p1, void *A, double *W, int64_t *counts, int *counts_phi,
                                  uint64_t *pair_total, void *stream);

/*
 * Fused histogram estimator for pivots [p0, p1): the multipoles of z3_accumulate_histogram
 * per pivot chunk, contracted as in z3_estimate (eq. zetamEst); zeta [m_max+1][nbins][nbins][2]
 * += (unnormalised), pair_total += pairs (may be NULL).  Both precisions keep the chunk's
 * multipoles in FP64 and contract them in FP64 (identical results): the pair walk and the
 * transform, FP64 on both, are the whole cost, and FP32 storage would reach ~1e-6 relative
 * error on noise-dominated high multipoles.
 */
z3_status z3_estimate_histogram(z3_index idx, int map, int m_max, int prec, int64_t p0, int64_t p1,
                                double *zeta, uint64_t *pair_total, void *stream);

/*
 * Multi-field estimator (the remark after eq. ubEstimator): three attached maps A, B, C of
 * one index (fields on the same positions and weights, e.g. several redshift bins of one
 * pixel grid).  The pivot carries field A, the bin b1 field B and the bin b2 field C:
 *   zeta[m][b1][b2] += sum_p w_p x^A_p X^B_m(b1; p) conj(X^C_m(b2; p))          (cyclic = 0)
 * or the sum of that term over the cyclic permutations (A;B,C) + (B;C,A) + (C;A,B)
 * (cyclic = 1).  Unnormalised like z3_estimate (divide by sum_p w_p, z3_finalize); the
 * result is not Hermitian unless B = C.  map_a, map_b, map_c in [0, nmaps); they may repeat.
 * The multipoles of each distinct field needed are computed once per pivot chunk: on the
 * FP64 path of a sky index, fields within one group of 4 attached maps (maps 4g..4g+3) share
 * one search pass; otherwise one search pass per field.  pair_total += pairs counted once.
 */
z3_status z3_estimate_cross(z3_index idx, int map_a, int map_b, int map_c, int cyclic, int m_max,
                            int prec, int64_t p0, int64_t p1, double *zeta, uint64_t *pair_total,
                            void *stream);

/*
 * One term of the multi-field estimator over distinct catalogues: pivots of catalogue A
 * (external arrays, as for z3_estimate_pivots) against neighbour catalogue B (idx_b, map
 * map_b) in bin b1 and neighbour catalogue C (idx_c, map_c) in bin b2:
 *   zeta[m][b1][b2] += sum_p w_p x_p X^B_m(b1; p) conj(X^C_m(b2; p))
 * each X the bin average of its own catalogue (eq. Xm.binned) around the pivot.  The two
 * indexes need identical bin edges and the same geometry (Z3_ERR_INVALID_ARG otherwise).
 *   piv_xyz [3][npiv] FP64 positions ([2][npiv] plane positions for planar indexes), of
 *           any length (see z3_estimate_pivots),
 *   piv_w [npiv] or NULL, piv_x [npiv]
 * pivots [p0, p1) are processed; pairs_b / pairs_c += the pairs with B / C (may be NULL);
 * sum_w[0] += the pivots' weights (may be NULL).  The cyclic sum over (A;BC), (B;CA),
 * (C;AB) is three calls with the roles rotated.  Unnormalised like z3_estimate.
 */
z3_status z3_estimate_cross_catalogues(z3_index idx_b, int map_b, z3_index idx_c, int map_c, int64_t npiv,
                                       const double *piv_xyz, const double *piv_w, const double *piv_x,
                                       int m_max, int prec, int64_t p0, int64_t p1, double *zeta,
                                       uint64_t *pairs_b, uint64_t *pairs_c, double *sum_w, void *stream);

/*
 * Fused estimator for ALL attached maps at once (many mock maps over one set of
 * positions, eqs. Xm.binned and zetamEst for each map): for every pair the bin test,
 * bearing and cos/sin(m phi) are computed once and applied to the values of all maps.
 * zeta [nmaps][m_max+1][nbins][nbins][2] += (unnormalised, one block per map, in map
 * order); pair_total += the number of pairs (counted once, not per map), or NULL.
 * One-map passes for 1 or 2 maps; up to 56 maps on the FP64 path and 24 on the mixed
 * path, one pass of the register-tiled kernel per group of 4 maps (3 or 4 maps per lane,
 * FP64 multipole sums), one or two maps left over in one-map passes.  More maps, or more than 4 maps with a block shape fixed by
 * z3_index_set_batch_shape: the per-pair harmonics of a group of 64 x (waves per block)
 * candidates form the B operand of MFMA products with the maps' values; FP64 path in FP64
 * MFMA, mixed path in FP32 MFMA with the FP32 sums added into FP64 every 128 candidates.
 * `prec` also selects the FP64 or the mixed (FP32 storage, split FP32 MFMA) contraction.
 * Synchronous on `stream` the first time an (m_max, prec) uses the MFMA kernel with an
 * automatic shape (the shapes are timed then), unless the stream is capturing.
 */
z3_status z3_estimate_maps(z3_index idx, int m_max, int prec, int64_t p0, int64_t p1,
                           double *zeta, uint64_t *pair_total, void *stream);

/*
 * Fused estimator for an external pivot catalogue against the index's neighbours (the
 * pivot field of the cross-correlation remark in the harmonic-decomposition section;
 * also the approximate search, whose neighbour catalogue is a coarsened map):
 *   piv_xyz  [3][npiv] FP64 positions ([2][npiv] positions for a planar index) in any
 *            order: each pivot chunk is sorted by the index's bands (a stable radix sort,
 *            256 cells per band) before its multipoles are formed, so an unordered
 *            catalogue runs as fast as a coherent one and repeated calls give identical
 *            results; only the order of the FP64 sum over pivots depends on the order
 *            given.  Normally unit vectors; a pivot of another
 *            length keeps the chord test on the raw vectors (its windows are rescaled),
 *            so pair lists match a direct evaluation of d2 on the same vectors
 *   piv_w    [npiv] pivot weights, or NULL for all 1
 *   piv_x    [npiv] pivot values
 * Pivots [p0, p1) are processed; zeta += sum_p w_p x_p X(b1) conj X(b2) (unnormalised),
 * pair_total += pairs (may be NULL), sum_w[0] += sum of the pivots' weights (may be NULL).
 * A neighbour at the position of a pivot is not a pair (E_0 > 0).
 */
z3_status z3_estimate_pivots(z3_index idx, int map, int64_t npiv, const double *piv_xyz,
                             const double *piv_w, const double *piv_x, int m_max, int prec,
                             int64_t p0, int64_t p1, double *zeta, uint64_t *pair_total,
                             double *sum_w, void *stream);

/*
 * Adjoint of the estimator for map `map` and pivots [p0, p1) (derived from eqs.
 * Xm.binned and zetamEst with the weights held fixed): for a real loss L and
 *   G [m_max+1][nbins][nbins][2] = (dL/dRe zeta, dL/dIm zeta),
 * where zeta = scale * sum_p w_p x_p X_p X_p^H over the given pivots,
 *   grad_x [n] += dL/dx  (catalogue order, FP64).
 * Pass scale = 1 / sum_p w_p for the normalised estimator.  The multipoles are recomputed
 * per pivot chunk; neighbour contributions are added with FP64 atomics, so the last bits
 * may vary between runs.  FP64 throughout.
 */
z3_status z3_adjoint(z3_index idx, int map, int m_max, int64_t p0, int64_t p1, const double *G,
                     double scale, double *grad_x, void *stream);

/*
 * Adjoint for ALL attached maps: G [nmaps][m_max+1][nbins][nbins][2], grad_x [nmaps][n] +=
 * (catalogue order), zeta of every map = scale * sum_p w_p x_p X_p X_p^H.  The multipoles
 * of several maps are recomputed together with shared pair geometry.
 */
z3_status z3_adjoint_maps(z3_index idx, int m_max, int64_t p0, int64_t p1, const double *G,
                          double scale, double *grad_x, void *stream);

/* sum_p w_p over pivots [p0, p1), FP64, out[0] += . */
z3_status z3_pivot_weight_sum(z3_index idx, int64_t p0, int64_t p1, double *out, void *stream);

/* zeta /= sum_w[0] for nmaps consecutive zeta arrays (the 1/sum_i w_i of eq. zetamEst). */
z3_status z3_finalize(int nmaps, int m_max, int nbins, double *zeta, const double *sum_w,
                      void *stream);

/*
 * Resummation (eq. eq_zeta_harmonic truncated at |m| <= m_max):
 *   out[b1][b2][k] = Re zeta_0 + 2 sum_{m=1}^{m_max} (Re zeta_m cos(m phi_k) - Im zeta_m sin(m phi_k))
 * phi [nphi] FP64 radians; out [nbins][nbins][nphi] FP64.
 */
z3_status z3_resum(int m_max, int nbins, const double *zeta, int nphi, const double *phi,
                   double *out, void *stream);

/*
 * FFTLog evaluation of the line-of-sight integrals of the modelling appendix ("FFTLog for
 * the line-of-sight integral"): the building blocks A_0, A_1, A_2 of the pre-cyclic model
 * 3PCF (eq. zetapc) for a batch of models that share the linear power spectrum and the
 * angle grid, each with its own line-of-sight kernel F(chi) = q_A q_B q_C D_+^4.
 *
 *   c_s     (eqs. pklfft, pklfft_eta, cm): N samples P(k_l), k_l = k_min (k_max/k_min)^{l/(N-1)},
 *           s = -N/2..N/2, eta_s = ((N-1)/N) 2 pi s / ln(k_max/k_min), end weights 1/2
 *   a_s     = 1 + nu + i eta_s, one bias nu per factor (n, mt):
 *           nu[0] (0,0), nu[1] (1,1), nu[2] (1,-1), nu[3] (2,0)
 *   g(a_s)  = 2^{mt+a_s-1} Gamma((1+mt+a_s+n)/2) / (pi Gamma((1-a_s-mt+n)/2))  (the Gamma-ratio
 *           form of the k integral)
 *   A_{s1 s2} = int dchi F(chi) chi^{-a_s1 - a_s2 - 2}: trapezoid rule in ln chi on the nchi
 *           points chi_j = chi_min (chi_max/chi_min)^{j/(nchi-1)}
 *   I^{(n1,mt1)}_{(n2,mt2)}(theta_i, theta_j) = sum_{s1,s2} c_s1 g1(a_s1) theta_i^{-(1+a_s1+mt1)}
 *           A_{s1 s2} c_s2 g2(a_s2) theta_j^{-(1+a_s2+mt2)}
 *   out[b][0] = A_0 = Re I^{(0,0)}_{(0,0)}, out[b][1] = A_1 = Re (I^{(1,1)}_{(1,-1)} + its
 *           transpose), out[b][2] = A_2 = Re I^{(2,0)}_{(2,0)}      (each [ntheta][ntheta])
 *
 *   N        even, 4 <= N <= Z3_MAX_FFTLOG_N;  Pk [N] FP64 samples of P_L on the k_l grid
 *   nu       [host] 4 biases, |nu| <= 50; a bias that puts a pole of either Gamma function
 *            on eta = 0 is Z3_ERR_INVALID_ARG
 *   F        [nmodels][nchi] FP64 kernel samples on the chi_j grid, nchi >= 2
 *   theta    [ntheta] FP64 angles in radians, > 0 (not checked: a non-positive angle gives
 *            non-finite outputs), 1 <= ntheta <= Z3_MAX_FFTLOG_THETA
 *   out      [nmodels][3][ntheta][ntheta] FP64, overwritten (not accumulated)
 *   workspace, workspace_bytes: device scratch of the caller, 256-byte aligned; NULL makes the library take it
 *            from its stream-ordered pool (at most 1 GiB; the call cannot then be captured
 *            into a graph).  z3_fftlog_workspace_size gives the bytes for a number of models
 *            per pass; a smaller workspace processes fewer models per pass (Z3_ERR_INVALID_ARG
 *            if it holds none).
 * Since eta_s is linear in s, A_{s1 s2} depends on s1 + s2 only: the library forms its
 * 2N + 1 distinct entries h(s1 + s2) (one product over chi for all models) and never the
 * (N+1)^2 matrix; since P is real, the terms (s1, s2) and (-s1, -s2) are conjugate and only
 * s1 >= 0 is summed (I = Re of twice that half, the s1 = 0 column once).  The products run on
 * FP64 matrix cores.  Everything is FP64; the results equal the dense-matrix evaluation up to
 * rounding (P and F must be real: they are FP64 arrays).
 */
#define Z3_MAX_FFTLOG_N 4096
#define Z3_MAX_FFTLOG_THETA 4096
z3_status z3_fftlog_workspace_size(int N, int nchi, int ntheta, int models_per_pass, size_t *bytes);
z3_status z3_fftlog_a_functions(int N, const double *Pk, double k_min, double k_max, const double *nu,
                                int nchi, double chi_min, double chi_max, int nmodels, const double *F,
                                int ntheta, const double *theta, double *out, void *workspace,
                                size_t workspace_bytes, void *stream);

/*
 * Largest single device allocation the library may make, in bytes (default: no limit; the
 * environment variable Z3_DEVICE_ALLOC_LIMIT_MB, read when the library is loaded, sets the
 * initial value).  A call that would need a larger buffer fails with Z3_ERR_OUT_OF_MEMORY
 * before it touches the device, exactly as when the device allocation itself fails: no
 * output written, no index created.  For callers that share a GPU, and for testing the
 * out-of-memory paths.  Applies to every thread and device; SIZE_MAX lifts it.
 */
z3_status z3_set_device_alloc_limit(size_t max_bytes);

/* Wait for the stream and report any asynchronous error. */
z3_status z3_sync(void *stream);

const char *z3_status_string(z3_status s);
const char *z3_last_error(void);

/*
 * Kernel timing for measurement: when enabled, the library brackets every launch of
 * its forward multipole kernels (one-map, register-tiled many-map, MFMA many-map and
 * angular-histogram) and of the chi-quadrature product of z3_fftlog_a_functions with HIP
 * events on the launch stream.  Launches made inside the adjoint calls and
 * calls on a stream that is being captured into a graph are not timed.  z3_profile_read
 * waits for those events and returns the number of launches and their summed duration.
 */
z3_status z3_profile_enable(int on);
z3_status z3_profile_read(int64_t *launches, double *total_ms, int reset);

#ifdef __cplusplus
}
#endif

#endif /* ZETA3_H */
