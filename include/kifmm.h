/*
 * kifmm.h -- C ABI of the MI355X kernel-independent FMM evaluation library.
 *
 * Computes the Laplace potential of Eq. (1) of the paper (section "The Fast
 * Multipole Method"),
 *
 *     phi_j = sum_{i : y_i != x_j} q_i / (4 pi |y_i - x_j|),
 *
 * at every target x_j due to every source y_i, with the kernel-independent
 * FMM: P2M, M2M, M2L (V list), P2L (X list), L2L, L2P, M2P (W list) and the
 * near field (U list) over an octree, on check and equivalent surfaces of
 * n_e = 6(p-1)^2 + 2 points (section "Computational structure of FMM
 * operators").  The evaluation runs on the current HIP device.
 *
 * Conventions for every entry point:
 *   - Return KIFMM_OK or an error status; on error, kifmm_last_error() holds
 *     a message for the calling thread and no output buffer has been written
 *     (except where stated).  No entry point aborts or throws.
 *   - The caller owns every buffer it passes.  The library never frees a
 *     caller buffer and keeps no caller pointer after returning.
 *   - Points are row-major [n][3] float64 host arrays.  Charges and
 *     potentials are row-major [n_rhs][n] arrays in the CALLER's order.
 *   - Trees and operator sets are opaque library-owned handles released by
 *     their *_destroy function.  A handle may be used from one thread at a
 *     time; calls that overlap on one handle race.
 */
#ifndef KIFMM_H
#define KIFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KIFMM_OK = 0,
  KIFMM_EINVAL = 1,       /* bad argument: null pointer, size, non-finite, range */
  KIFMM_ENOMEM = 2,       /* host or device allocation failed */
  KIFMM_EDEVICE = 3,      /* a HIP runtime call failed (message has its text) */
  KIFMM_EUNSUPPORTED = 4  /* valid request the library does not implement */
} kifmm_status;

/* Arithmetic of an evaluation.  In every mode the check-to-equivalent solves
 * (UC2E, DC2E) run in FP64 and the per-target sum of near and far field is
 * accumulated in FP64.  In the FP32-bulk modes the equivalent-surface terms
 * (L2P, M2P) are computed in FP64 from order p >= 10 (tuning key
 * "far_fp64_min_p"). */
typedef enum {
  KIFMM_FP64 = 0,        /* every operator in FP64 */
  KIFMM_FP32 = 1,        /* particle operators, M2M, L2L, M2L in FP32 */
  KIFMM_M2L_BF16X3 = 2,  /* as FP32; M2L as A_h x_h + A_h x_l + A_l x_h, BF16
                            MFMA products accumulated in FP32 */
  KIFMM_M2L_BF16X5 = 3,  /* as FP32; M2L with the density split three ways:
                            A_h x_h + A_h x_m + A_l x_h + A_l x_m + A_h x_l */
  KIFMM_M2L_F16X3 = 4,   /* as FP32; M2L as A_h x_h + A_h x_l + A_l x_h in FP16
                            (11-bit significands) on MFMA, FP32 accumulation;
                            operators and densities scaled by powers of two
                            into FP16 range, so the scaling is exact */
  KIFMM_FP64_M2L_FP32 = 5,  /* every operator in FP64 except M2L (FP32 MFMA) */
  KIFMM_FP64_M2L_F16X3 = 6  /* every operator in FP64 except M2L (split FP16 as
                               in KIFMM_M2L_F16X3) */
} kifmm_precision;

/* Octree parameters (section "Computational structure of FMM operators":
 * n_crit is the leaf capacity; the 2:1 balance condition).  All geometric
 * decisions are taken in FP64:
 *   root: (root_center, root_halfwidth) if root_halfwidth > 0, else the
 *     bounding cube of all points, centre (min+max)/2, half-width
 *     max extent/2 * (1 + 2^-20);
 *   level-l box index of a point: clamp(floor(t * 2^l), 0, 2^l - 1) per axis,
 *     t = (x - (c0 - r0)) / (2 r0). */
typedef struct {
  int32_t uniform_depth; /* >= 0: uniform tree, every non-empty box split down to
                            this level; -1: adaptive tree */
  int32_t ncrit;         /* adaptive: split a box holding more than ncrit sources
                            or more than ncrit targets (>= 1) */
  int32_t max_depth;     /* adaptive: deepest level, 0..20 */
  int32_t balance;       /* adaptive: 1 = enforce 2:1 balance between touching
                            leaves (face, edge or corner), 0 = off */
  double root_center[3];
  double root_halfwidth; /* > 0 to fix the root cube; 0 = derive from the points */
} kifmm_tree_params;

typedef struct kifmm_tree kifmm_tree;
typedef struct kifmm_ops kifmm_ops;

/* Summary of a built tree (counts of interaction-list entries over all boxes). */
typedef struct {
  int64_t n_src, n_tgt;
  int32_t depth, n_boxes, n_leaves, reserved;
  int64_t n_u, n_v, n_w, n_x;
  double root_center[3];
  double root_halfwidth;
} kifmm_tree_info;

/* Build the octree and the U, V, W, X interaction lists on the host.
 * src_xyz [n_src][3], tgt_xyz [n_tgt][3]: host FP64, finite; n_src, n_tgt >= 1.
 * tgt_xyz may alias src_xyz (then self-interaction is excluded, Eq. 1).
 * The device copy is made on first use by an evaluate call, on the device that
 * is current then.  EINVAL on bad input, ENOMEM on allocation failure. */
kifmm_status kifmm_build_tree(const double* src_xyz, int64_t n_src,
                              const double* tgt_xyz, int64_t n_tgt,
                              const kifmm_tree_params* params, kifmm_tree** out);

/* The same tree built on the current GPU (section "Data-oriented design of
 * PyExaFMM": linear octree of Morton-sorted points; lists of section
 * "Computational structure of FMM operators"): root, keys, stable sort,
 * refinement, 2:1 balance, numbering and the U, V, W, X lists run as
 * kernels, and the result is equal, integer for integer (keys, point order,
 * boxes, lists), to kifmm_build_tree on the same coordinates; the host copy
 * is filled from the device.  src_xyz [n_src][3], tgt_xyz [n_tgt][3]: DEVICE
 * FP64 (tgt_xyz == src_xyz with n_tgt == n_src: the same points, as in
 * kifmm_build_tree).  Work is ordered on hip_stream (NULL: the default
 * stream), which is synchronised before return.  Errors as
 * kifmm_build_tree, plus EINVAL for host pointers; EUNSUPPORTED past the
 * device scan limit (about 8M boxes on one level). */
kifmm_status kifmm_build_tree_device(const double* src_xyz, int64_t n_src,
                                     const double* tgt_xyz, int64_t n_tgt,
                                     const kifmm_tree_params* params, void* hip_stream,
                                     kifmm_tree** out);

kifmm_status kifmm_tree_get_info(const kifmm_tree* tree, kifmm_tree_info* info);

/* Copy the box table out (for inspection and tests).  Boxes are numbered
 * level by level, Morton order within a level.  Every pointer may be NULL to
 * skip that array; otherwise it must hold n_boxes entries ([n_boxes][3] for
 * anchor, [n_boxes][2] for the half-open ranges into the sorted points). */
kifmm_status kifmm_tree_export_boxes(const kifmm_tree* tree, int32_t* level,
                                     int32_t* anchor, int32_t* parent,
                                     int32_t* is_leaf, int64_t* src_range,
                                     int64_t* tgt_range);

/* Copy one interaction list out as CSR over boxes: which = 0 U, 1 V, 2 W, 3 X.
 * offsets [n_boxes + 1]; items [offsets[n_boxes]] box ids (may be NULL to
 * query the size through offsets only).  Lists skip source boxes that hold no
 * source (their contribution is zero). */
kifmm_status kifmm_tree_export_list(const kifmm_tree* tree, int32_t which,
                                    int64_t* offsets, int32_t* items);

/* Sorted-to-caller permutations: src_perm[i] is the caller index of the i-th
 * sorted source (either pointer may be NULL). */
kifmm_status kifmm_tree_export_perm(const kifmm_tree* tree, int64_t* src_perm,
                                    int64_t* tgt_perm);

/* Re-sort new positions of the tree's points on the GPU (the part of the
 * tree build that depends on the points: the linear octree of section
 * "Data-oriented design" keeps points sorted by the Morton key of their leaf,
 * boxes as ranges of that order).  While every point stays in a leaf that
 * held points of its kind (sources, targets) before and no such leaf
 * empties, boxes, interaction lists and evaluation plans are unchanged; the
 * sorted order, the leaf-relative coordinates and the box ranges are
 * recomputed on the device with the host build's rules (keys at the tree's
 * key level from its root cube, clamped at its faces; a stable sort, ties in
 * caller order).  Uniform trees then equal kifmm_build_tree on the new
 * points with the same root, bit for bit; so do adaptive trees whose fresh
 * build would refine the same way (no leaf crossing n_crit), and otherwise
 * they keep their boxes, which remains a valid FMM tree for the new points.
 * src_xyz: device FP64 [n_src][3], n_src as built.  tgt_xyz: device FP64
 * [n_tgt][3]; NULL if the tree was built with tgt_xyz == src_xyz (the targets
 * are the sources).  hip_stream: stream the work runs on (NULL: default); the
 * call synchronises it.  A tree evaluated on this device takes the new order
 * in place (its plans and a captured graph stay valid); the host copy
 * (exports, new plans) is refreshed on first use.
 * Errors: EINVAL (null tree, host pointers, missing targets, or a point in a
 * leaf cell that held no point of its kind before, or an occupied leaf left
 * empty: the tree is unchanged; build a new tree), EDEVICE. */
kifmm_status kifmm_tree_update_points(kifmm_tree* tree, const double* src_xyz,
                                      const double* tgt_xyz, void* hip_stream);

/* Precompute the operators of order p (2 <= p <= 16) on the host in FP64:
 * surfaces, UC2E/DC2E pseudo-inverses truncated at rcond * sigma_max
 * (0 < rcond < 1), the 8 M2M and 8 L2L child operators and the 316 M2L
 * offset operators, on a reference box; per-level scaling is applied in the
 * evaluation (section "Parallelization strategies for FMM operators").
 * The device copy is made on first use. */
kifmm_status kifmm_precompute_operators(int32_t p, double rcond, kifmm_ops** out);

/* kifmm_precompute_operators with options.  flags: 0, or
 * KIFMM_PRECOMPUTE_DEVICE_SVD: the two check-to-equivalent pseudo-inverses
 * (the dominant cost: an n x n SVD each, n = 488 at p = 10) are computed on
 * the current GPU with rocSOLVER's FP64 SVD and the same truncation rule;
 * they agree with the host's one-sided Jacobi result to the conditioning of
 * the kept singular values (~1e-9 relative), not bitwise.  Synchronises the
 * device.  EINVAL for an unknown flag; EDEVICE if the GPU SVD fails. */
#define KIFMM_PRECOMPUTE_DEVICE_SVD 1
kifmm_status kifmm_precompute_operators_ex(int32_t p, double rcond, int32_t flags,
                                           kifmm_ops** out);

/* Operators of the screened (Yukawa) kernel exp(-kappa r) / (4 pi r),
 * kappa > 0: the method is kernel independent (its operators are kernel
 * evaluations on the check and equivalent surfaces and pseudo-inverses of
 * them; section "Computational structure of FMM operators"), but this kernel
 * is not homogeneous, so one set of tables is formed per level l = 2 ..
 * max_level for boxes of half-width root_halfwidth / 2^l (the Laplace
 * kernel's single reference set does not apply).  The operators serve trees
 * with exactly that root half-width and depth <= max_level (evaluate returns
 * EINVAL otherwise); kifmm_evaluate and kifmm_evaluate_batch use the kernel
 * in every step (the particle kernels evaluate exp(-kappa r) / r), and so
 * does kifmm_evaluate_gradient (-(1 + kappa r) exp(-kappa r) (x - y) / r^3);
 * the operator cache is Laplace-only (EUNSUPPORTED).  flags as in
 * kifmm_precompute_operators_ex.  EINVAL for kappa <= 0, root_halfwidth <= 0
 * or max_level outside [2, 20]. */
kifmm_status kifmm_precompute_operators_screened(int32_t p, double rcond, double kappa,
                                                 double root_halfwidth, int32_t max_level,
                                                 int32_t flags, kifmm_ops** out);

/* Persistent operator cache.  kifmm_ops_save writes every table of `ops`
 * with its key (p, rcond, the surface radii 1.05 / 2.95) and a checksum to
 * `path` (through a temporary file renamed into place).  kifmm_ops_load
 * reads it back, bitwise equal, if the file holds operators of exactly
 * (p, rcond) and is intact; otherwise EINVAL with the reason (missing,
 * foreign or damaged file, other key), and *out is untouched. */
kifmm_status kifmm_ops_save(const kifmm_ops* ops, const char* path);
kifmm_status kifmm_ops_load(const char* path, int32_t p, double rcond, kifmm_ops** out);

/* Copy an operator table out (tests): which = 0 surface [n][3], 1 UC2E [n][n],
 * 2 DC2E [n][n], 3 M2M [8][n][n], 4 L2L [8][n][n], 5 M2L [316][n][n],
 * 6 M2L offsets [316][3] (as doubles).  Row-major, reference box of
 * half-width 1.  n_out is the number of doubles `out` can hold. */
kifmm_status kifmm_ops_export(const kifmm_ops* ops, int32_t which, double* out,
                              int64_t n_out);
int32_t kifmm_ops_n(const kifmm_ops* ops); /* surface points n, or -1 */
/* Table sets of `ops`: 1 (Laplace kernel), or max_level + 1 (screened kernel:
 * kifmm_ops_export then returns every table as [levels][...], set l for
 * boxes of half-width root_halfwidth / 2^l, sets 0 and 1 zero); -1 for NULL. */
int32_t kifmm_ops_levels(const kifmm_ops* ops);

/* Evaluate the potentials (one hipGraph replay on a non-default stream, see
 * the "graph" tuning key).  charges: DEVICE [n_rhs][n_src] (caller order),
 * potentials: DEVICE [n_rhs][n_tgt] (caller order), both FP64 if
 * io_fp64 != 0, else FP32.  n_rhs >= 1.  Runs asynchronously on hip_stream
 * (a hipStream_t; NULL = the default stream); inputs must stay valid and
 * unmodified until the stream reaches the end of the work.  The first call
 * for a (tree, ops, precision, n_rhs) allocates and uploads device state that
 * is reused by later calls. */
kifmm_status kifmm_evaluate(const kifmm_tree* tree, const kifmm_ops* ops,
                            const void* charges, int32_t n_rhs, void* potentials,
                            int32_t io_fp64, kifmm_precision precision,
                            void* hip_stream);

/* kifmm_evaluate for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * It calls no hipMalloc, hipFree or allocating library routine: every work
 * buffer of the evaluation (gathered charges, check potentials, equivalent
 * densities, split M2L operand, pair products, FP64 sums) is carved from a
 * fixed device array of 256 MiB that each GPU running the library holds until
 * the process ends, and the kernels are launched eagerly on hip_stream (no
 * graph of its own, so a caller may capture the call).  Same arguments,
 * layouts, ownership and results (bitwise) as kifmm_evaluate.
 * Preconditions: one kifmm_evaluate of (tree, ops, n_rhs, precision) on the
 * current device since the tree, its points (kifmm_tree_update_points) or
 * the tuning last changed, so that the tree's device state and the operator
 * tables are resident; otherwise EINVAL.  EUNSUPPORTED if the work buffers
 * exceed 256 MiB (the message gives the size needed; 1M points at p = 6 in
 * the FP32-bulk modes need ~140 MiB); EINVAL while phase profiling is on.
 * Every call on one GPU uses that GPU's array: calls that overlap on one GPU
 * (other streams, other threads) race and must be ordered by the caller. */
kifmm_status kifmm_evaluate_noalloc(const kifmm_tree* tree, const kifmm_ops* ops,
                                    const void* charges, int32_t n_rhs, void* potentials,
                                    int32_t io_fp64, kifmm_precision precision,
                                    void* hip_stream);

/* Potentials and their gradients at the targets (the derivative of Eq. (1)
 * in the target position; the paper evaluates potentials only).  The
 * multipole passes are those of kifmm_evaluate; the leaf stage (L2P, M2P,
 * near field) also applies the kernel's derivative to the same densities and
 * charges.  out: DEVICE [n_rhs][4][n_tgt] (caller order): component 0 the
 * potential, 1..3 d/dx, d/dy, d/dz; FP64 if io_fp64 != 0, else FP32.  Other
 * arguments, stream semantics and errors as kifmm_evaluate.  In the FP32-bulk
 * precisions the downward pass runs L2L and DC2E in FP64 here (the gradient
 * amplifies FP32 rounding noise on the downward check surface): the potential
 * component then agrees with kifmm_evaluate's result to that mode's accuracy,
 * in FP64 to rounding. */
kifmm_status kifmm_evaluate_gradient(const kifmm_tree* tree, const kifmm_ops* ops,
                                     const void* charges, int32_t n_rhs, void* out,
                                     int32_t io_fp64, kifmm_precision precision,
                                     void* hip_stream);

/* Evaluate n_prob independent problems (each its own tree, n_rhs = 1) in one
 * pass: every operator runs as one launch over all problems.  charges[k],
 * potentials[k]: device buffers of problem k, as in kifmm_evaluate.  The
 * trees are treated as one forest and its device state is cached for the
 * same ordered set of tree handles. */
kifmm_status kifmm_evaluate_batch(int32_t n_prob, const kifmm_tree* const* trees,
                                  const kifmm_ops* ops, const void* const* charges,
                                  void* const* potentials, int32_t io_fp64,
                                  kifmm_precision precision, void* hip_stream);

/* Whole pipeline from host arrays: build an adaptive tree (ncrit 64, balanced),
 * precompute order p with rcond 1e-9, evaluate in FP32 (precision KIFMM_FP32),
 * copy the FP64 potentials back.  Synchronous.  src, q [n_src]; tgt, pot
 * [n_tgt]; host memory. */
kifmm_status kifmm_evaluate_simple(const double* src, const double* q, int64_t n_src,
                                   const double* tgt, int64_t n_tgt, int32_t p,
                                   double* pot);

/* Per-phase device timing of evaluate calls: when enabled, each phase of every
 * later evaluate is bracketed by HIP events on the evaluation stream and its
 * duration accumulated.  Phase names: kifmm_phase_name(i), i < kifmm_n_phases().
 * kifmm_get_phase_times fills ms[i] (total milliseconds) and launches[i]
 * (number of kernel launches of phase i), and resets the counters.  It
 * synchronises the stream of the last evaluate. */
kifmm_status kifmm_set_profiling(int32_t enable);
int32_t kifmm_n_phases(void);
/* Number of evaluation graphs captured so far in this process (an evaluate
 * on a non-default stream captures one when the tree's last graph was made
 * for another precision, stream, operator set, buffers or tuning, and
 * replays it otherwise).  An operator set made after another was destroyed
 * never replays the other's graph, even at the same address.  Never fails. */
int64_t kifmm_graph_captures(void);

/* Test hook for the out-of-memory paths: after `after` more allocation
 * points of the library succeed (host tree, plan and operator builds, every
 * device allocation), the next one fails as an allocation would, with
 * KIFMM_ENOMEM, and the hook disarms itself; after < 0 disarms it.  A call
 * that fails this way leaves its handles and cached state as they were
 * before the call.  Process-wide; not for production use. */
void kifmm_debug_fail_allocations(int64_t after);
const char* kifmm_phase_name(int32_t i);
kifmm_status kifmm_get_phase_times(double* ms, int64_t* launches);

/* Copy an intermediate buffer of the last kifmm_evaluate on `tree` to the host
 * as FP64 (inspection and per-operator tests).  which = 0 upward check
 * potentials, 1 upward equivalent densities, 2 downward check potentials,
 * 3 downward equivalent densities (each [n_boxes][n_rhs][n], box order of
 * kifmm_tree_export_boxes, check potentials scaled by the box half-width),
 * 4 potentials [n_rhs][n_tgt] in sorted target order.  fp64 and n_rhs select
 * the cached evaluation (precision FP64 or not).  Synchronises the device.
 * EINVAL if no such evaluation has run or n_out is too small. */
kifmm_status kifmm_debug_buffer(const kifmm_tree* tree, int32_t which, int32_t fp64,
                                int32_t n_rhs, double* out, int64_t n_out);

/* Process-wide tuning knobs of the evaluation kernels (a change of a plan
 * knob rebuilds the plans at the next evaluate).
 *   "m2l_tile_cols":  output columns (box x right-hand side) per M2L tile,
 *                     64 (default), 96, 128, 160 or 192.  Above 128, M2L kernels
 *                     with 32-bit outputs run one 768-thread block per tile
 *                     (split modes up to 160 columns: the kernel of
 *                     m2l_async); the others cover the tile with 64-column
 *                     slices.  Results are bitwise equal to those of
 *                     64-column tiles.
 *   "far_fp64_min_p": smallest order p at which FP32-bulk modes evaluate the
 *                     equivalent-surface terms in FP64 (default 10; 2..17,
 *                     17 = never).
 *   "m2l_check_min_p": smallest order p at which the FP32 and split-FP16 M2L
 *                     act on upward check potentials with the operators
 *                     folded with UC2E (M2L_o * UC2E, formed in FP64) instead
 *                     of on equivalent densities (default 10; 17 = never).
 *   "graph":          1 (default): an evaluation on a non-default stream is
 *                     captured into a hipGraph on first use and replayed with
 *                     one launch while tree, operators, precision, stream and
 *                     buffers are unchanged (profiling runs eagerly); 0: eager.
 *   "m2l_fp64_sum_min_p": smallest order p at which an M2L that accumulates
 *                     in FP32 (FP32, BF16 and FP16 products) moves its sums
 *                     into FP64 after every operator step (default 10; 17 =
 *                     never).
 *   "m2l_pair_fill":  percent, default 40.  A problem whose M2L tiles would
 *                     be less full than this (V-list pairs over 64 tile
 *                     columns x the union of the tile's offsets: adaptive
 *                     trees of surfaces) runs M2L pair by pair instead: tiles
 *                     of pairs that share one offset write each product to a
 *                     pair buffer (n_pairs x n_rhs x ld values, ld = n
 *                     rounded up to 32, allocated on the first evaluation),
 *                     then each target sums its pairs in offset order.  The
 *                     percentage applies at ld = 160 (p = 6) and scales with
 *                     sqrt(ld / 160).  Decided per problem, so batches and
 *                     multi-RHS runs match single runs bitwise, unless the
 *                     pair buffer would pass 64 GiB (then every problem of
 *                     that evaluation runs gathered tiles).  0: never;
 *                     101: always (within the cap).
 *   "m2l_split":      1 (default): every M2L tile runs as two blocks, one for
 *                     the offsets with even x component and one for the odd,
 *                     both adding into the zeroed output with atomics; each
 *                     output is then the sum of two terms, so results stay
 *                     bitwise reproducible.  0: one block per tile.
 *   "m2l_wide":       1: split-BF16 and split-FP16 M2L plans of 65..128
 *                     columns (m2l_tile_cols 128) run a kernel whose waves
 *                     own 80 x 64 outputs and take the densities from global
 *                     memory straight into registers; 0 (default): the
 *                     general gathered-GEMM kernel.  Results are bitwise
 *                     equal.
 *   "m2l_async":      1 (default): split-BF16 and split-FP16 M2L plans of
 *                     up to 160 columns (m2l_tile_cols 64, 128, 160; the
 *                     gathered tiles and the pair tiles; with FP64 sums, see
 *                     m2l_fp64_sum_min_p, up to 96 columns in blocks of 128
 *                     operator rows, else 64) run a kernel that
 *                     stages operator and density chunks from global memory
 *                     straight into LDS, two chunks in flight; 0: the
 *                     general gathered-GEMM kernel (and, with m2l_wide, the
 *                     wide-tile kernel).  Results are bitwise equal.
 *   "m2l_rows":       operator rows per M2L block: 160, 128, or 0 (default)
 *                     for the one that pads the operator's rows (n rounded
 *                     up to 32) the least: 128 at p = 4, 5, 7, 10.  Results
 *                     are bitwise equal.
 *   "near_fork":      4 (default): near field (P2P) and far field (L2P,
 *                     M2P) of each leaf are summed by one kernel at the end
 *                     of the evaluation.  0..3: the near field runs as its
 *                     own kernel on a second stream, forked after the points
 *                     are gathered (0), after P2M (2), before M2L (1) or
 *                     after M2L (3), and joins before the far field.
 * EINVAL for an unknown key or value. */
kifmm_status kifmm_set_tuning(const char* key, int32_t value);

/* The value a tuning knob of kifmm_set_tuning currently holds (its default
 * until it is set), written to *value.  Process-wide, like the knobs; the
 * autotuner (paper_2303_08394_amd/autotune.py) reads the layout keys before
 * it searches them.  EINVAL for a null argument or an unknown key. */
kifmm_status kifmm_get_tuning(const char* key, int32_t* value);

void kifmm_tree_destroy(kifmm_tree* tree);
void kifmm_ops_destroy(kifmm_ops* ops);

/* Message of the last non-OK status returned to the calling thread. */
const char* kifmm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KIFMM_H */
