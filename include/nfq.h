/*
 * nfq.h -- C ABI of the near-field quadrature-correction generator for
 * layer potentials on surfaces made of curved triangular patches.
 *
 * Method: Greengard, O'Neil, Rachh, Vico, "Fast multipole methods for the
 * evaluation of layer potentials with locally-corrected quadratures"
 * (arXiv 2006.02545).  For every target x and every patch Gamma_j of the
 * dual list T_eta(x) (Section 4, near-field definitions), and for the
 * target's own patch when the target is a discretisation node (self
 * interaction, start of Section 4), the library computes the weights
 *
 *     a^j_l(x) = sum_{nm} V_(nm),l I^j_nm(x),                    (Section 4.3)
 *     I^j_nm(x) = int_T0 Kern(x, X^j(u,v)) K_nm(u,v) du dv,
 *     Kern = alpha G_k(r) J + beta n(y).grad_y G_k(x, y),        (Sections 1, 3)
 *
 * n = X_u x X_v (unnormalised), J = |n|, G_k = e^{ikr}/(4 pi r), K_nm the
 * orthonormal Koornwinder polynomials on T0 and V the values-to-coefficients
 * matrix of the patch's interpolation nodes (Section 2).  Near pairs use the
 * adaptive 1->4 midpoint subdivision of Section 4.3; self pairs use a
 * target-split, Duffy-collapsed tensor Gauss-Legendre rule standing in for the
 * generalised Gaussian tables of Section 4.  The weights are returned as one
 * sparse matrix in CSR-by-target order (storage of the near and self
 * matrices, Section 5.2): row t holds, in ascending patch order, the blocks of
 * every patch of T_eta(x_t) and of the target's own patch; inside a block the
 * patch's nodes in order; column = global node id.
 *
 * Conventions
 *  - Degree d means polynomials of total degree <= d, n_d = (d+1)(d+2)/2
 *    nodes per patch (the paper's order p = d + 1).  Supported d: 1..8.
 *  - All array arguments of nfq_plan_create / nfq_generate / nfq_apply /
 *    nfq_adjoint are DEVICE pointers on the context's device, borrowed for
 *    the duration of the enqueued work; the caller owns them and must keep
 *    them alive until the stream has passed the work.  Host pointers are
 *    marked "host".
 *  - Every call enqueues on the context's stream (the hipStream_t given to
 *    nfq_create) and returns without synchronising, except where noted.
 *  - Return codes: 0 = NFQ_OK, > 0 warnings (results written), < 0 errors
 *    (nothing usable written).  No C++ exception crosses the ABI.  Errors
 *    detected on the device surface at the next synchronising call
 *    (nfq_plan_create, nfq_generate with a stats pointer, nfq_sync).
 *    nfq_last_error returns a message for the last error on a context.
 */
#ifndef NFQ_H
#define NFQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nfq_status;

#define NFQ_OK 0
#define NFQ_WARN_NONCONVERGED 1     /* some near pairs hit max_depth; values written */
#define NFQ_ERR_INVALID_ARG (-1)
#define NFQ_ERR_NOT_REGISTERED (-2) /* a patch uses a degree not registered */
#define NFQ_ERR_DEGENERATE_PATCH (-3)
#define NFQ_ERR_SINGULAR_PAIR (-4)  /* a near target coincides with a patch point */
#define NFQ_ERR_OUT_OF_MEMORY (-5)
#define NFQ_ERR_HIP (-6)
#define NFQ_ERR_UNSUPPORTED (-7)

typedef struct nfq_ctx nfq_ctx;
typedef struct nfq_plan nfq_plan;

/* Patches (Section 3.1): patch j has degree[j] and its n_d nodes are
 * xyz[node_ptr[j] .. node_ptr[j+1]) in the order of the registered
 * reference nodes of that degree.  Device arrays. */
typedef struct {
    int64_t P;
    const int32_t *degree;   /* [P] */
    const int64_t *node_ptr; /* [P+1], node_ptr[j+1] - node_ptr[j] = n_{degree[j]} */
    const double *xyz;       /* [N][3], N = node_ptr[P] */
} nfq_surface;

/* Targets (Section 5.2): points x_t; node_of_target[t] is the global node id
 * when the target is a discretisation node (then its own patch's self block
 * is generated) or -1 for an off-surface target.  Device arrays. */
typedef struct {
    int64_t NT;
    const double *xyz;             /* [NT][3] */
    const int64_t *node_of_target; /* [NT] */
} nfq_targets;

/* Dual near lists T_eta(x_t) (Section 4): CSR by target, patch ids strictly
 * ascending in each row, the target's own patch excluded.  Device arrays. */
typedef struct {
    const int64_t *row_ptr; /* [NT+1] */
    const int32_t *patch;   /* [row_ptr[NT]] */
} nfq_nearlist;

/* Kernel alpha S_k + beta D_k (Section 3: single layer, double layer; the
 * combined field D - ik S is alpha = -ik, beta = 1).  Complex wavenumber
 * allowed (Im k >= 0).  k = 0 with real alpha, beta gives real weights. */
typedef struct {
    double alpha_re, alpha_im;
    double beta_re, beta_im;
    double k_re, k_im;
} nfq_kernel;

/* Parameters.  tol = requested precision eps (Section 4.2-4.3); the adaptive
 * test is ||I_T - sum I_children||_2 <= loosen * eps * d_j / ||V||_2 *
 * |T|/|T0| (loosen = 1 reproduces the paper's bound; the paper sets the
 * termination eps "somewhat larger", loosen > 1).  max_depth bounds the
 * subdivision (pairs reaching it are counted as non-converged).
 * ng: points per direction of the subtriangle rule (0 = default 8; only 8 is
 * supported).  self_nr / self_na: radial / angular Gauss-Legendre sizes of
 * the self rule per panel, at most 64 (0 = per-degree defaults: 10 / 16 for
 * degree <= 3, 14 / 20 for 4, 16 / 24 for 5, 18 / 28 for 6 and 7, 20 / 32
 * for 8). */
typedef struct {
    double tol;
    double loosen;
    int32_t max_depth;
    int32_t ng;
    int32_t self_nr;
    int32_t self_na;
    int32_t flags;  /* bit 0 (NFQ_FLAG_TIMING): time each phase with HIP events
                       on the context's stream, reported in nfq_stats;
                       bit 1 (NFQ_FLAG_PER_PAIR): use the plain per-pair near
                       kernel (one wavefront per pair, no reuse of subtriangle
                       geometry across targets) instead of the patch-centric one */
    int32_t min_depth; /* subdivide at least this deep (0: adaptive from the
                          root); min_depth = max_depth gives uniform trees,
                          whose weights are smooth in the geometry */
} nfq_params;

#define NFQ_FLAG_TIMING 1
#define NFQ_FLAG_PER_PAIR 2

typedef struct {
    int64_t near_pairs;
    int64_t self_pairs;
    int64_t visits;        /* subtriangle rule evaluations (near pairs) */
    int64_t checks;        /* parent-vs-children tests */
    int64_t nonconverged;  /* near pairs that reached max_depth */
    int64_t max_level;     /* deepest subdivision level used */
    /* phase durations in ms (NFQ_FLAG_TIMING only, else 0): pair builder,
     * patch preparation, self quadrature, adaptive near quadrature,
     * moments -> weights */
    double ms_builder, ms_prep, ms_self, ms_near, ms_weights;
} nfq_stats;

/* Create a context on HIP device `device` bound to stream `hip_stream`
 * (a hipStream_t; NULL = the default stream).  *out receives the context. */
nfq_status nfq_create(int device, void *hip_stream, nfq_ctx **out);
void nfq_destroy(nfq_ctx *ctx);

/* Register reference nodes for degree d (Section 2.1: the interpolation nodes
 * on T0, the paper's Vioreanu-Rokhlin nodes).  ref_uv: host [n_d][2] (u, v),
 * strictly inside T0.  ref_w: host [n_d] quadrature weights or NULL for the
 * interpolatory weights w_l = int_T0 L_l.  Builds U, V = U^{-1}, ||V||_2 on
 * the host and uploads them.  Errors: INVALID_ARG (node outside T0, or the
 * nodes are not unisolvent: cond(U) > 1e12), UNSUPPORTED (d outside 1..8). */
nfq_status nfq_register_degree(nfq_ctx *ctx, int d, const double *ref_uv, const double *ref_w);

/* Size the correction matrix for a surface, target set and near list.
 * Fills the caller-allocated device array row_ptr[NT+1] (CSR row pointers of
 * the output) and *nnz_out (host) with its number of entries; the plan owns
 * its scratch.  Synchronises the stream.  The plan keeps the pointers of
 * surf/targets/near: the arrays must stay valid (their contents may change
 * between nfq_generate calls as long as the near-list structure and the
 * degrees do not).  Errors: INVALID_ARG (sizes, unsorted rows, own patch in
 * a near row, bad node ids), NOT_REGISTERED, OUT_OF_MEMORY, HIP_ERROR. */
nfq_status nfq_plan_create(nfq_ctx *ctx, const nfq_surface *surf, const nfq_targets *targets,
                           const nfq_nearlist *near, nfq_plan **out, int64_t *nnz_out,
                           int64_t *row_ptr);

/* Generate the correction matrix: pair/work-queue build, patch preparation,
 * adaptive near quadrature, self quadrature, moments -> node weights, column
 * indices.  col: device int32[nnz]; val: device [nnz] double (real kernels:
 * k = 0 and real alpha, beta) or interleaved complex128 (re, im) otherwise.
 * stats: host or NULL; when given, the call synchronises, fills it and
 * returns NFQ_WARN_NONCONVERGED if any near pair reached max_depth. */
nfq_status nfq_generate(nfq_plan *plan, const nfq_kernel *kern, const nfq_params *params,
                        int32_t *col, void *val, nfq_stats *stats);

/* y = A sigma with the generated matrix (the local-correction part of the
 * subtract-and-add apply, Section 5.3).  val, sigma [N], y [NT]: device,
 * same value type as val (complex128 interleaved or double). */
nfq_status nfq_apply(nfq_plan *plan, const int32_t *col, const void *val, const void *sigma,
                     void *y);

/* Adjoint (gradient) of Phi = sum_t conj(lambda_t) (A sigma)_t for the
 * quadrature nfq_generate computes with the same kernel and parameters: the
 * adaptive decisions are recomputed, then the quadrature sum over the
 * accepted subtriangles (and the self rules, with their split points and
 * grading held fixed) is differentiated.  sigma: device complex128 [N]
 * (nodal density), lambda: device complex128 [NT].  Outputs (device,
 * complex128, interleaved): grad_xyz [N][3] = dPhi/dx_node (chart nodes, plus
 * the target position for node targets; each node may be the target of at
 * most one target), grad_k [1] = dPhi/dk at fixed alpha, beta, and dphi_dab
 * [2] = (dPhi/dalpha, dPhi/dbeta) or NULL.  Deterministic.  Not part of the
 * paper (a companion for shape optimisation and inverse problems).
 * Errors: as nfq_generate; UNSUPPORTED when near pairs on degree-7 patches are
 * present (that kernel instance is disabled: it returned non-finite values). */
nfq_status nfq_adjoint(nfq_plan *plan, const nfq_kernel *kern, const nfq_params *params,
                       const void *sigma, const void *lambda, void *grad_xyz, void *grad_k,
                       void *dphi_dab);

/* Wait for all work enqueued on the context's stream; reports device-side
 * errors of earlier calls. */
nfq_status nfq_sync(nfq_ctx *ctx);

/* Near lists T_eta(x_t) on the device (near-field definitions of Section 4;
 * lists by target, Section 5.2), in the nfq_nearlist layout that
 * nfq_plan_create takes.  Patch j's ball has centre c_j = parametric mean of
 * the chart, (1/|T0|) int_T0 X^j du dv, and radius R_j = max |X^j(u,v) - c_j|
 * over the lattice (i/64, k/64), i + k <= 64, of T0; target t is near patch
 * j when |x_t - c_j| < eta R_j and j is not the target's own patch.
 * Arguments: surf, targets as for nfq_plan_create (device arrays; the
 * degrees must be registered); eta > 0; row_ptr: caller-allocated device
 * int64 [NT+1], always written on success and on the capacity error;
 * patch: caller-allocated device int32 [capacity] (may be NULL when capacity
 * is 0), rows strictly ascending; *nnz_out (host): number of near pairs;
 * centres [P][3], radii [P]: device outputs or NULL.  When nnz exceeds
 * capacity nothing is written to patch and the call returns
 * NFQ_ERR_INVALID_ARG with *nnz_out set: call again with capacity >= nnz.
 * Allocates its scratch and frees it before returning; synchronises the
 * stream.  Deterministic.  Errors: INVALID_ARG (sizes, eta, null arrays,
 * non-finite targets, capacity), NOT_REGISTERED, OUT_OF_MEMORY, HIP_ERROR. */
nfq_status nfq_near_lists(nfq_ctx *ctx, const nfq_surface *surf, const nfq_targets *targets,
                          double eta, int64_t *row_ptr, int32_t *patch, int64_t capacity,
                          int64_t *nnz_out, double *centres, double *radii);

void nfq_plan_destroy(nfq_plan *plan);
const char *nfq_status_str(nfq_status s);
const char *nfq_last_error(nfq_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* NFQ_H */
