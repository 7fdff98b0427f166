/*
 * wqa.h -- C ABI of the weighted-quadrature assembly library (libwqa.so) for MI355X.
 *
 * The library assembles, row by row, the isogeometric mass matrix
 *     M_ij = integral of c B_i B_j                                   (eq:Mass)
 * and stiffness matrix with a diagonal coefficient A = diag(a_1..a_d)
 *     K_ij = integral of sum_k a_k dB_i/dx_k dB_j/dx_k               (eq:Stiffness)
 * on the open uniform tensor-product B-spline space of degree p in {2, 3}
 * (C^1 quadratic, C^2 cubic) and dimension d in {2, 3} (Sec. 2.2, eq:Gmap2,
 * eq:Gmap3), with the geometry already folded into c and a_k (eq:PullBacks).
 * Row i is integrated with its own weighted Gaussian rule whose weight function is
 * B_i (eq:GaussQuadSys for the mass terms, eq:GaussQuadSysStiff for the stiffness
 * terms), one direction at a time (eq:Decompo), into the (2p+1)^d band of row i
 * (Fig. 1).  It also evaluates the adjoint of both maps.
 *
 * Vocabulary and layouts (all C order):
 *   n_k       = N_el,k + p basis functions in direction k (eq:DimUni); rows = prod n_k.
 *   Q         = p + 1 quadrature nodes per row per direction (one per element of the
 *               row's support for interior rows, Sec. 3).
 *   S         = 2p + 1 band slots per direction; slot s_k of row i holds column
 *               j_k = i_k - p + s_k (Fig. 1).
 *   Row i     = (i_1..i_d), flat index ((i_1 n_2) + i_2) n_3 + i_3 (d = 3).
 *   Matrix    = [rows][S^d] values ("structured CSR": the column pattern is implicit).
 *               Slots whose column leaves [0, n_k) in some direction are written 0.
 *   Grid      = [N_1..N_d] samples, N_k = n_k Q.  The mass coefficient c lives on the
 *               grid whose direction-k coordinates are the mass-rule nodes of every
 *               row (row i owns points (i_k Q + q_k)_k).  a_k lives on the grid that
 *               uses the stiffness-rule nodes in direction k and mass-rule nodes in
 *               the other directions.  wqa_get_rules returns those coordinates.
 *               Sample buffers (c, a_k, f, dc, da_k) hold a grid in this layout, with
 *               lines optionally padded (wqa_set_grid_pitch), or the same samples row
 *               by row, [rows][Q^d] (wqa_set_sample_layout); "[N_1..N_d]" below stands
 *               for whichever layout is set.
 *
 * Alignment: every device buffer (coefficients, matrices, gradients) must start on a
 * 16-byte boundary (hipMalloc and PyTorch allocations do); WQA_EINVAL otherwise.
 *
 * Ownership: every device buffer passed in belongs to the caller; the library owns
 * the context and its (small) rule tables on host and device.  The assemble calls
 * never allocate, run asynchronously on the given HIP stream (NULL = default
 * stream) and return as soon as the work is queued.  A context is not thread-safe;
 * use one per host thread.
 *
 * Errors: every call returns a wqa_status; on failure wqa_last_error() gives a
 * thread-local message.  Device faults surface at the caller's next synchronization.
 * Inputs must be finite; non-finite samples propagate into the rows that read them.
 */
#ifndef WQA_H
#define WQA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WQA_ABI_VERSION 1

typedef struct wqa_ctx wqa_ctx;

typedef enum wqa_status {
    WQA_OK = 0,
    WQA_EINVAL = -1,        /* bad argument (null pointer, out-of-range value) */
    WQA_ESTATE = -2,        /* call out of order (no space / no rules / no device) */
    WQA_EUNSUPPORTED = -3,  /* degree or dimension without rules (p not in {2,3}, d not in {2,3}) */
    WQA_ERULE = -4,         /* a rule table failed validation, or a rule could not be solved */
    WQA_EHIP = -5,          /* HIP runtime error (message carries hipGetErrorString) */
    WQA_ENOMEM = -6         /* host or device allocation failed */
} wqa_status;

typedef enum wqa_dtype { WQA_F32 = 0, WQA_F64 = 1 } wqa_dtype;

typedef enum wqa_kind { WQA_MASS = 0, WQA_STIFFNESS = 1 } wqa_kind;

/* How the last directional contraction (the final pass, over the first direction)
 * accumulates in the FP32 mode; every other stage accumulates in FP32 and every input,
 * output and intermediate stays FP32.  FP64 calls always accumulate in FP64.  Both
 * non-plain variants return the final pass's sum as if it had been computed in at
 * least twice the working precision and rounded once to FP32. */
typedef enum wqa_final {
    WQA_FINAL_PLAIN = 0,  /* FP32 fused multiply-adds */
    WQA_FINAL_DOT2 = 1,   /* compensated summation in FP32 registers: error-free products
                             (FMA) and error-free sums, the errors summed apart and added
                             once (Ogita, Rump, Oishi's Dot2) */
    WQA_FINAL_F64 = 2     /* mixed precision, not compensated: each FP32 stage result is
                             multiplied by the FP64 table entry of the first direction and
                             the products are summed in an FP64 register, rounded once to
                             FP32 (default; products and sums round at 2^-53) */
} wqa_final;

/* Returns WQA_ABI_VERSION of the loaded library. */
int wqa_abi_version(void);

/* Message of the last failing call on this thread ("" if none).  The pointer stays
 * valid until the next library call on the same thread. */
const char *wqa_last_error(void);

/* Creates a context on HIP device hip_device (>= 0), or a host-only context when
 * hip_device == -1 (space, rules and tables work; the assemble calls return
 * WQA_ESTATE).  *out receives the context; destroy it with wqa_destroy. */
wqa_status wqa_create(wqa_ctx **out, int hip_device);

/* Frees the context and its device tables (after synchronizing its device).  NULL is ignored. */
void wqa_destroy(wqa_ctx *ctx);

/* Sets the spline space: dimension dim in {2, 3}, degree in {2, 3}, n_elem[dim]
 * elements per direction (each in [degree + 1, 2^24]; WQA_EINVAL otherwise), open
 * uniform knots on [0, 1] (eq:Gmap3).  Discards any rules set before. */
wqa_status wqa_set_space(wqa_ctx *ctx, int dim, int degree, const int64_t *n_elem);

/* Sets the knots of direction dir to the open knot vector with breakpoints
 * breaks[0..n_elem[dir]] (0 = b_0 < b_1 < ... < b_N = 1; p+1 fold ends, simple interior
 * knots, eq:Gmap3), or back to uniform when breaks is NULL.  Discards that direction's
 * rules; wqa_set_default_rules then traces every row's rule from the uniform one by
 * homotopy continuation of the knots (the approach the paper names for its future work,
 * Sec. 1 and Conclusion), and wqa_set_rules validates against these knots.  WQA_EINVAL
 * for breakpoints that do not run from 0 to 1 or are not strictly increasing. */
wqa_status wqa_set_knots(wqa_ctx *ctx, int dir, const double *breaks);

/* Installs the default rules for both kinds in every direction: the paper's
 * interior rules (eq:WQquadratic, eq:WQcubic, eq:WQquadraticStiff, eq:WQcubicStiff),
 * solved on the host by Newton (x87 extended precision, rounded once to FP64) from
 * the exactness conditions, translated to
 * every interior row; and, for the p rows at each end that the paper leaves open
 * (Remark closing Sec. 3.2), weighted Gaussian rules of at most p+1 nodes solved the
 * same way (exactness on the row's interacting functions, completed by degree-
 * elevation monomials), padded to Q nodes with zero weights.  On a direction with
 * breakpoints (wqa_set_knots) each row's rule is traced from that uniform rule along
 * the straight path of the knots; the free parameter that symmetry fixes on uniform
 * knots is fixed by the condition symmetry leaves in the elements' own coordinates.
 * WQA_ERULE when a path meets a singular point (a stiffness node reaching the zero of
 * B'_j, where its weight diverges): there is no rule of this family on those knots. */
wqa_status wqa_set_default_rules(wqa_ctx *ctx);

/* Installs a caller's rule for one kind and direction: nodes[n_dir*q] in [0, 1] and
 * weights[n_dir*q], row-major by row j then node, q == degree + 1.  The weights
 * multiply the product of both functions, i.e. the rule claims
 *     integral phi_i phi_j dx  ~=  sum_m weights[j*q+m] phi_i(x_m) phi_j(x_m)
 * with phi = B (WQA_MASS) or phi = dB/dx (WQA_STIFFNESS) in parametric units
 * (eq:GaussQuadSys, eq:GaussQuadSysStiff).  When exact_tol >= 0 every row is
 * validated: nodes with nonzero weight lie strictly inside supp(B_j) and at least
 * 1e-9 element widths from any knot, and the relative exactness residual over the
 * interacting columns is <= exact_tol (WQA_ERULE otherwise, nothing installed).
 * exact_tol < 0 skips validation.  Any order of a row's nodes is accepted (the grid
 * coordinates follow it); the kernels skip table entries that vanish for rules with one
 * node per support element in order, and take the full loops in a direction whose
 * rules break that pattern.  Nodes in FP64 parametric units carry up to
 * n_elem * 2^-53 element widths of rounding, so no rule shows a residual much below
 * that on long directions (wqa_set_default_rules validates its own rules against
 * max(1e-12, 8 n_elem 2^-53)).  Copies the arrays; uploads the tables to the device of
 * a device context.
 *
 * Ordering: the calls that change rules or knots (wqa_set_rules, wqa_set_default_rules,
 * wqa_set_space, wqa_set_knots followed by either) wait for every kernel queued on the
 * context's device, on any stream, before they touch the device tables; work queued
 * before such a call uses the old rules, work queued after it the new ones. */
wqa_status wqa_set_rules(wqa_ctx *ctx, wqa_kind kind, int dir, int q,
                         const double *nodes, const double *weights, double exact_tol);

/* Copies the rule in use for (kind, dir) into nodes[n_dir*q] and weights[n_dir*q]
 * (either may be NULL).  The nodes are the grid coordinates of direction dir for
 * every field that uses that kind of rule in that direction. */
wqa_status wqa_get_rules(const wqa_ctx *ctx, wqa_kind kind, int dir, double *nodes, double *weights);

/* Copies the FP64 contraction table of (kind, dir): out[n_dir][q][S] with
 * out = weight * phi_j(x) * phi_{j-p+s}(x) at node x of row j (0 for columns
 * outside the space).  This is what the kernels contract with. */
wqa_status wqa_get_tables(const wqa_ctx *ctx, wqa_kind kind, int dir, double *out);

/* Sizes of the current space (any pointer may be NULL): rows, S^d slots per row,
 * Q^d points per row, grid_dims[dim] = N_k. */
wqa_status wqa_query(const wqa_ctx *ctx, int64_t *n_rows, int64_t *slots_per_row,
                     int64_t *points_per_row, int64_t *grid_dims);

/* Selects how FP32 calls accumulate the final directional pass (default WQA_FINAL_F64). */
wqa_status wqa_set_final_mode(wqa_ctx *ctx, wqa_final mode);

/* Sets the distance, in values, between consecutive grid lines of the last direction in
 * every grid-shaped buffer the calls read or write (c, a_k, f, dc, da_k): such a buffer
 * then holds N_1 x .. x N_{d-1} lines of `pitch` values, whose first N_d values are the
 * grid (Grid above) and whose rest is never read or written.  0 restores the dense
 * layout (pitch N_d, the default).  Otherwise pitch must be a multiple of 4 and at least
 * N_d (WQA_EINVAL).  A pitch that is a multiple of 32 (FP32) or 16 (FP64) values starts
 * every grid line on a 128-byte boundary of a 128-byte aligned buffer, so that the
 * adjoint writes each line's gradient runs as whole cache lines.  wqa_set_space resets
 * it; WQA_ESTATE before a space is set. */
wqa_status wqa_set_grid_pitch(wqa_ctx *ctx, int64_t pitch);

/* Layouts of the sample buffers (c, a_k, f, dc, da_k). */
typedef enum wqa_samples {
    WQA_SAMPLES_GRID = 0,  /* [N_1..N_d], Grid above (the default) */
    WQA_SAMPLES_ROWS = 1   /* [rows][Q^d]: the Q^d points that row i owns, (i_k Q + q_k)_k,
                              as one block at offset i Q^d (row order as for the matrices),
                              point (q_1..q_d) at ((q_1 Q) + q_2) Q + q_3 (d = 3) or
                              q_1 Q + q_2 (d = 2) within it */
} wqa_samples;

/* Selects the layout of every sample buffer the calls read or write (c, a_k, f, dc,
 * da_k).  Both layouts hold the same values: each grid point belongs to exactly one row,
 * the row whose rule it is a node of (Sec. 3), and WQA_SAMPLES_ROWS stores the Q^d samples
 * of each row together, rows in order.  Every result is the same, bit for bit, in both
 * layouts.  In the row layout a tile of consecutive rows reads (assembly, products) and
 * writes (adjoint) its samples of a field as one contiguous block, which the adjoint
 * writes with whole-block 16-byte stores.  wqa_set_space resets it to WQA_SAMPLES_GRID.
 * WQA_EINVAL for other values; WQA_ESTATE before a space is set, or for WQA_SAMPLES_ROWS
 * while a grid pitch is set (the pitch belongs to the grid layout; wqa_set_grid_pitch
 * likewise refuses a nonzero pitch in the row layout). */
wqa_status wqa_set_sample_layout(wqa_ctx *ctx, int layout);

/* Caps the wave tasks (tiles of consecutive rows) one kernel dispatch takes: launches
 * with more are queued as several dispatches on the same stream, with identical
 * results.  0 restores the default, 2^24 tasks, which keeps every dispatch below HIP's
 * 32-bit work-item count whatever the space (a 2D quadratic space of 2^24 x 64 elements
 * needs about 10^8 tasks); larger values are clamped to it.  WQA_EINVAL for negative
 * values. */
wqa_status wqa_set_dispatch_limit(wqa_ctx *ctx, int64_t max_tasks);

/* Mass matrix (eq:Mass with the folded coefficient c).  c: device [N_1..N_d] of dtype
 * on the all-mass grid; M: device [rows][S^d] of dtype (fully overwritten). */
wqa_status wqa_assemble_mass(wqa_ctx *ctx, wqa_dtype dtype, const void *c, void *M,
                             void *hip_stream);

/* Stiffness matrix (eq:Stiffness with the folded diagonal coefficient).  a[dim]:
 * device pointers, a[k] on the grid with the stiffness rule in direction k;
 * K: device [rows][S^d] (fully overwritten). */
wqa_status wqa_assemble_stiffness(wqa_ctx *ctx, wqa_dtype dtype, const void *const *a,
                                  void *K, void *hip_stream);

/* Both matrices in one pass over the rows (same arguments as the two calls above). */
wqa_status wqa_assemble_fused(wqa_ctx *ctx, wqa_dtype dtype, const void *c,
                              const void *const *a, void *M, void *K, void *hip_stream);

/* Adjoint: with L = <gM, M> + <gK, K> (sums over every slot), writes dc = dL/dc and
 * da[k] = dL/da_k at every grid point.  gM, gK: device [rows][S^d]; slots outside the
 * space are ignored (may hold anything).  gM == NULL skips dc (dc must be NULL then);
 * gK == NULL skips da (da must be NULL then).  Each grid point belongs to exactly
 * one row, so every output element is written once, without atomics. */
wqa_status wqa_assemble_adjoint(wqa_ctx *ctx, wqa_dtype dtype, const void *gM,
                                const void *gK, void *dc, void *const *da,
                                void *hip_stream);

/* Load vector (eq:Load): b_i = integral f B_i over the unit square or cube, with the mass
 * rules.  Since the basis functions sum to one, f B_i = sum_j f B_i B_j, so b is the
 * vector of row sums of the mass matrix assembled with c = f, and every row rule that is
 * exact for M is exact here.  f: device [N_1..N_d] of dtype on the all-mass grid (like c);
 * b: device [rows] of dtype (fully overwritten). */
wqa_status wqa_assemble_load(wqa_ctx *ctx, wqa_dtype dtype, const void *f, void *b, void *hip_stream);

/* Matrix-free product y = M x with the mass matrix of coefficient c (eq:Mass, eq:LinSys):
 * y_i = sum_j M_ij x_j with the same rules, tables and samples as wqa_assemble_mass, but
 * M is never formed: x is contracted with the tables to every row's own points, direction
 * by direction (eq:Decompo; in 3D once per block of neighbouring rows, each partial sum
 * shared by the rows whose bands contain it), multiplied by c there and summed over each
 * row's points.  Results equal sum_j M_ij x_j up to rounding order.  c as in wqa_assemble_mass;
 * x, y: device [rows] of dtype (x is read, y fully overwritten; they must not overlap).
 * Arithmetic is plain in the dtype (no compensated final pass). */
wqa_status wqa_apply_mass(wqa_ctx *ctx, wqa_dtype dtype, const void *c, const void *x, void *y,
                          void *hip_stream);

/* Matrix-free product y = K x with the stiffness matrix of the diagonal coefficient a
 * (eq:Stiffness), as wqa_apply_mass; a as in wqa_assemble_stiffness. */
wqa_status wqa_apply_stiffness(wqa_ctx *ctx, wqa_dtype dtype, const void *const *a, const void *x,
                               void *y, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* WQA_H */
