/*
 * libhinv — hierarchical-inverse EMT network solver for AMD MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only.  "Host" arguments are CPU memory
 * that the library copies during the call (the caller may free them on
 * return).  "Device" arguments are HIP device memory owned by the caller.
 * A stream argument is a hipStream_t passed as void* (NULL = the null
 * stream).  Every call returns a hinv_status; hinv_last_error() gives a
 * message for the last non-OK status of the calling thread.  No call throws
 * or aborts across this boundary.  One handle must not be used from two
 * threads at once.
 *
 * The paper (Zhang et al., "An Efficient Network Solver for EMT Simulation
 * ... Hierarchical Inverse Computation and Modification") defines:
 *   - the network equation G v(t) = i_in(t) + i_his(t - dt), real values
 *     (Section II, Eq. (1)); its inverse-based solution v = G^{-1} i (Eq. (2));
 *   - a partition tree whose nodes own bus sets, leaves being small
 *     sub-networks (Section III.B, Fig. 2-3); the inverse of each node's
 *     diagonal block is built from its children's inverses and a low-rank
 *     coupling H = h_l h_r^T over the cut lines (Eq. (9), Algorithm 1);
 *   - the update of G^{-1} when a line between buses i and j changes
 *     (Section IV, Algorithm 2).
 * This library keeps that structure but stores the exact inverse: at each
 * tree node the coupling level is a Woodbury capacitance matrix
 * S = C + U^T B^{-1} U over the cut lines (the paper's M of Eq. (8)-(9) is
 * this form with S truncated to C, available as hinv_options.coupling =
 * HINV_COUPLING_PAPER).  A line change is applied either as a
 * Sherman-Morrison-Woodbury low-rank correction of the stored inverse
 * (hinv_modify_line, and the line losses of the EMT time loop) or as a local
 * rebuild of the stored inverse itself (hinv_update_line, Algorithm 2 made
 * exact).  emt_network3_csr gives the three-phase G of a network and
 * emt3_create its time loop; chol_* is a sparse Cholesky network solution kept
 * as a comparison baseline.
 */
#ifndef HINV_H
#define HINV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HINV_OK = 0,
    HINV_E_INVALID = 1,        /* bad argument; nothing was launched */
    HINV_E_NOT_SPD = 2,        /* a leaf block is not positive definite, or a change makes G indefinite */
    HINV_E_NO_MEMORY = 3,      /* workspace smaller than hinv_workspace_size / emt_workspace_size */
    HINV_E_DEVICE = 4,         /* a HIP runtime call failed */
    HINV_E_NO_SUCH_LINE = 5,   /* the line to change does not exist (or has less conductance) */
    HINV_E_NO_CONVERGENCE = 6, /* iterative refinement did not reach rel_tol in max_refine steps */
    HINV_E_RANK_LIMIT = 7,     /* more line changes than max_mod_rank */
    HINV_E_SINGULAR = 8        /* a coupling (capacitance) matrix is singular */
} hinv_status;

/* Storage / arithmetic precision of the stored inverse blocks used by the
 * per-step apply.  FP64 applies in FP64.  The others apply in that storage
 * precision with FP32 accumulation and recover FP64 accuracy by iterative
 * refinement against the sparse G in FP64. */
typedef enum { HINV_FP64 = 0, HINV_FP32 = 1, HINV_BF16 = 2, HINV_FP8 = 3 } hinv_precision;

typedef struct hinv_ctx* hinv_handle;
typedef struct emt_ctx* emt_handle;

/* Symmetric sparse matrix, full pattern (both triangles), 0-based, FP64,
 * column indices sorted within a row.  Host memory. */
typedef struct {
    int32_t n;
    const int32_t* row_ptr;   /* [n+1] */
    const int32_t* col_idx;   /* [row_ptr[n]] */
    const double* val;        /* [row_ptr[n]] */
} hinv_csr;

/* Partition tree (Section III.B).  parent[k] is the parent of node k, -1 for
 * the single root; a node's children are the nodes naming it as parent, in
 * index order.  bus_leaf[a] is the leaf that owns bus a; every leaf owns at
 * least one bus and at most HINV_MAX_LEAF buses; internal nodes own the union
 * of their children.  Host memory. */
typedef struct {
    int32_t n_nodes;
    const int32_t* parent;    /* [n_nodes] */
    const int32_t* bus_leaf;  /* [n] */
} hinv_tree;

#define HINV_MAX_LEAF 128

typedef struct {
    int32_t prec;          /* hinv_precision of the per-step apply */
    double rel_tol;        /* refinement stop: ||dv||_inf <= rel_tol * ||v||_inf (mixed precision or
                              HINV_COUPLING_PAPER only) */
    int32_t max_refine;    /* refinement iterations after the first apply (mixed precision or
                              HINV_COUPLING_PAPER only) */
    int32_t max_mod_rank;  /* line changes a handle (or each case) can hold, 0..16 */
    int32_t max_nrhs;      /* largest nrhs passed to hinv_solve (>= 1) */
    int32_t warm_start;    /* EMT, FP32/BF16/FP8 storage, every engine: max_refine + 1 corrections
                              per step starting from the previous step's v instead of P b plus
                              max_refine corrections.  FP64 storage, every engine: the incremental form
                              v = v_prev + P (b - G v_prev), one FP64 apply per step (max_refine and
                              rel_tol unused); equal to P b in exact arithmetic, it keeps rounding from
                              accumulating along a mode the step map does not damp (a bus whose only
                              line is lost keeps its voltage on its shunt capacitor); serving takes the
                              pool's warm_start the same way. */
    int32_t kernel_mode;   /* EMT engine: 0 = automatic (one case: 3, else 5, when it fits;
                              several cases: 4 when it fits; else 2 when it fits, else 1); 1 = one
                              launch per kernel per step (any size); 2 = one fused launch per
                              emt_step, one workgroup per case (case vectors in LDS); 3 = one fused
                              cooperative launch per emt_step, one workgroup per leaf of a single
                              case, every coupling level in every workgroup's LDS; 4 = fused
                              cooperative launches, cases in panels of 16 with one workgroup per
                              leaf per panel, leaf blocks applied to a panel as one matrix-core
                              product (max_mod_rank <= 2); 5 = one fused cooperative launch, one
                              workgroup per leaf of a single case, coupling levels computed by the
                              owners of their columns with a barrier per exchange (trees too large
                              for 3).  Engines 1 and 3-5 run exactly max_refine (+1 when
                              warm-started) corrections per step in mixed precision */
    int32_t coupling;      /* hinv_coupling: HINV_COUPLING_EXACT stores the exact inverse;
                              HINV_COUPLING_PAPER stores the paper's approximation (Algorithm 1 as
                              printed: every capacitance inverse S^{-1} replaced by C, i.e. each
                              node's off-diagonal blocks M = -G_i^{-1} H_ij G_j^{-1} of Eq. (8) built
                              from the children's approximations); hinv_solve then runs max_refine
                              FP64-residual corrections in any precision.  hinv_build only: the EMT
                              and serving entry points need the exact inverse (HINV_E_INVALID) */
} hinv_options;

typedef enum { HINV_COUPLING_EXACT = 0, HINV_COUPLING_PAPER = 1 } hinv_coupling;

typedef struct {
    int64_t n, n_leaves, n_internal, n_levels, n_cols;
    int64_t leaf_entries, z_entries, s_entries;   /* stored FP64 entries of each kind */
    int64_t max_leaf, max_cols;                   /* largest leaf, largest coupling level (2 x cut lines) */
    double apply_flops;   /* one FP64 apply G^{-1} x: 2 nl^2 per leaf; per node m (gather) + 2 m^2 (S^{-1});
                             2 pn pm per Z panel */
    double build_flops;   /* the build: 2 nl^3 per leaf elimination; per Z column the leaf column and the
                             updates of its ancestors below the node; m^2 per S assembly; 2 m^3 per S
                             inversion */
} hinv_info_t;

/* ---- Hierarchical inverse of a conductance matrix ---------------------- */

/* Device workspace bytes hinv_build needs for this matrix, tree and options.
 * Validates the inputs (symmetry, index ranges, tree shape, leaf sizes). */
hinv_status hinv_workspace_size(const hinv_csr* G, const hinv_tree* tree, const hinv_options* opt,
                                size_t* bytes);

/* Build the exact hierarchical inverse of G (Algorithm 1, exact coupling
 * levels) in FP64 on the GPU: leaf-block inverses, then per tree level the
 * panels Z = B^{-1} U and the inverses of the capacitance matrices S; then
 * the low-precision copies.  d_ws: device workspace of ws_bytes bytes
 * (>= hinv_workspace_size), owned by the caller, must outlive the handle and
 * must not be shared with another handle.  Synchronises the stream before
 * returning so that HINV_E_NOT_SPD / HINV_E_SINGULAR can be reported. */
hinv_status hinv_build(const hinv_csr* G, const hinv_tree* tree, const hinv_options* opt,
                       void* d_ws, size_t ws_bytes, void* stream, hinv_handle* out);

/* Apply a change of delta_g siemens to the line between buses a and b
 * (b = -1: between a and ground), i.e. G <- G + delta_g (e_a - e_b)(e_a - e_b)^T
 * (Section IV; the paper's "loss of a line" is delta_g = -g).  The stored
 * inverse gets a rank-1 Sherman-Morrison-Woodbury correction: u = G^{-1} w is
 * computed by one FP64 apply and the small capacitance matrix is inverted in
 * FP64.  Later solves use the changed G (also in refinement residuals).
 * Errors: HINV_E_INVALID (indices), HINV_E_NO_SUCH_LINE (delta_g < 0 larger
 * than the conductance between a and b), HINV_E_RANK_LIMIT, HINV_E_NOT_SPD
 * (the change makes G indefinite).  Synchronises the stream. */
hinv_status hinv_modify_line(hinv_handle h, int32_t a, int32_t b, double delta_g, void* stream);

/* What hinv_update_line rebuilt. */
typedef struct {
    int32_t lca_level;   /* tree level of the ends' lowest common ancestor (0: both ends in one leaf) */
    int32_t leaves;      /* leaf-block inverses recomputed (1 or 2) */
    int32_t columns;     /* coupling columns Z recomputed */
    int32_t nodes;       /* capacitance inverses S^{-1} recomputed */
} hinv_update_info;

/* Change the base matrix itself by the same line change, G <- G + delta_g
 * (e_a - e_b)(e_a - e_b)^T, and rebuild in FP64 only the part of the stored
 * inverse that the change reaches (Section IV, Algorithm 2: the leaf blocks of
 * a and b are re-inverted and the coupling data along their paths to the tree
 * root is recomputed; the column pair of a line between two leaves gets its new
 * weight at their lowest common ancestor).  Nodes above that ancestor are
 * recomputed too, so the result is the exact inverse of the new G: for a change
 * that leaves G's nonzero pattern intact it equals a fresh hinv_build of the
 * new G bit for bit.  Changes stored by hinv_modify_line stay in force on top
 * of the new base (their vectors are recomputed).  b = -1: between a and ground.
 * The entry (a, b) must exist in G, and a line between two leaves must be one
 * of the tree's coupling lines (nonzero in the built G; once set to zero by an
 * update it keeps its column with weight 0), else HINV_E_NO_SUCH_LINE.  The new
 * off-diagonal G[a][b] - delta_g must stay <= 0 (HINV_E_NO_SUCH_LINE).
 * HINV_E_NOT_SPD / HINV_E_SINGULAR: the new G is not positive definite, or the
 * stored changes become singular on it; the previous inverse is restored
 * exactly.  out (host, may be NULL) receives what was rebuilt.  Synchronises
 * the stream. */
hinv_status hinv_update_line(hinv_handle h, int32_t a, int32_t b, double delta_g, void* stream,
                             hinv_update_info* out);

/* v = G^{-1} i for nrhs right-hand sides (Eq. (2)).  d_i, d_v: device FP64,
 * column k at offset k*ld, rows in the caller's bus order; d_i and d_v may
 * not overlap.  nrhs <= opt.max_nrhs, ld >= n.  Asynchronous on the stream;
 * device-side failures surface through hinv_sync_status. */
hinv_status hinv_solve(hinv_handle h, const double* d_i, double* d_v, int32_t nrhs, int32_t ld,
                       void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as hinv_solve, bit for bit, with its per-call temporaries (permuted
 * input and output, level values, refinement residual and correction,
 * convergence stats) in the library's static device scratch instead of the
 * handle's workspace, so nrhs is not bounded by opt.max_nrhs.  Allocates
 * nothing and calls no allocating routine.  The scratch is 32 MiB per GPU,
 * held from the first hinv_build on that device until the process ends; a call
 * needs 8 * nrhs * (4n + n_cols) bytes plus 256-byte alignment per part
 * (n_cols: coupling columns of the tree, hinv_get_info), and a larger request
 * fails with HINV_E_INVALID before any launch.  Every call on one GPU shares
 * that GPU's scratch, which keeps the last call's contents: calls that overlap
 * in time on one GPU (on different streams or threads) race and must be
 * serialised by the caller.  Arguments, layout and errors as hinv_solve. */
hinv_status hinv_solve_noalloc(hinv_handle h, const double* d_i, double* d_v, int32_t nrhs, int32_t ld,
                               void* stream);

/* What hinv_solve_gmres did. */
typedef struct {
    int32_t corrections;       /* outer corrections (FP64 residual + GMRES solve + update) */
    int32_t inner_iterations;  /* GMRES iterations summed over the corrections (each one applies M, i.e. the
                                  stored inverse once and G `smooth` times, and G once to every column) */
    double last_update;        /* max over columns of ||d||_inf / ||x||_inf of the last correction */
} hinv_gmres_info;

/* Device workspace of hinv_solve_gmres for nrhs columns and at most m GMRES
 * iterations per correction (1 <= m <= 64): about 8 n nrhs (2m + 7) bytes. */
hinv_status hinv_gmres_workspace_size(hinv_handle h, int32_t nrhs, int32_t m, size_t* bytes);

/* v = G^{-1} i (Eq. (2)) to FP64 accuracy when the stored inverse is too
 * coarse for plain refinement (BF16 or scaled FP8 storage, whose apply error
 * makes the refinement of hinv_solve converge slowly or diverge): GMRES-based
 * iterative refinement with the preconditioner M = the stored inverse P applied
 * in its storage precision (with the stored line changes, as in hinv_solve),
 * followed by `smooth` (0..16) damped-Jacobi sweeps z += (2/3) D^{-1} (v - G z),
 * D = diag(G): a coarse stored inverse errs most where G amplifies, at high
 * frequencies, which these sweeps damp.  x_0 = M i.  Each correction:
 * r = i - G x in FP64 with the sparse G (and the stored changes); d ~ G^{-1} r
 * by flexible GMRES in FP64 on G M (right preconditioned; classical
 * Gram-Schmidt applied twice; Givens rotations), stopped once every column's
 * residual estimate is <= inner_tol ||r|| or after m iterations; x += d.  Stops
 * when max ||d||_inf / ||x||_inf <= rel_tol or after max_outer corrections
 * (then HINV_E_NO_CONVERGENCE, with the iterate written).  Vectors and layout
 * as hinv_solve (no bound by opt.max_nrhs); d_ws: device workspace of
 * hinv_gmres_workspace_size(h, nrhs, m) bytes, caller-owned, contents
 * overwritten.  0 < inner_tol < 1, rel_tol > 0, max_outer >= 0.  info (host,
 * may be NULL) receives the counts.  The host decides when to stop from one
 * small device-to-host copy per GMRES iteration, so the call synchronises the
 * stream. */
hinv_status hinv_solve_gmres(hinv_handle h, const double* d_i, double* d_v, int32_t nrhs, int32_t ld, int32_t m,
                             int32_t max_outer, int32_t smooth, double inner_tol, double rel_tol, void* d_ws,
                             size_t ws_bytes, void* stream, hinv_gmres_info* info);

/* After the caller has synchronised the stream: HINV_E_NO_CONVERGENCE or
 * HINV_E_NOT_SPD if a kernel flagged it since the last call, else HINV_OK.
 * Clears the flags. */
hinv_status hinv_sync_status(hinv_handle h);

/* Sizes and FLOP counts of the stored inverse (host memory out). */
hinv_status hinv_get_info(hinv_handle h, hinv_info_t* out);
/* Frees the handle (the caller still owns the workspace); NULL is accepted. */
hinv_status hinv_destroy(hinv_handle h);

/* ---- Comparison baseline: sparse Cholesky network solution -------------- */

/* Not the paper's method: the sparse direct solution it replaces (the LU-based
 * solver of the Introduction and Section V.B; G is SPD, so Cholesky).  The
 * factorization runs on the host (minimum-degree ordering, elimination tree,
 * up-looking Cholesky); the two triangular solves run on the GPU, one
 * workgroup per call, level by level (one barrier per level), x in LDS. */
typedef struct chol_ctx* chol_handle;

typedef struct {
    int64_t n, nnz_l;            /* order; stored entries of L (diagonal included) */
    int64_t fwd_levels, bwd_levels;   /* levels of the forward / backward solve */
    double solve_flops;          /* per right-hand side: 4 (nnz_l - n) + 2 n */
    double factor_flops;         /* of the numeric factorization */
} chol_info_t;

/* Device workspace for G (n <= 16384); factorizes on the host to size it.
 * Errors: HINV_E_INVALID, HINV_E_NOT_SPD (a pivot <= 0). */
hinv_status chol_workspace_size(const hinv_csr* G, size_t* bytes);
/* Factorize G and upload L and the level schedules into d_ws (caller-owned,
 * >= chol_workspace_size bytes, must outlive the handle).  Synchronises. */
hinv_status chol_create(const hinv_csr* G, void* d_ws, size_t ws_bytes, void* stream, chol_handle* out);
/* x = G^{-1} b for nrhs right-hand sides, one after the other in one launch;
 * column k at offset k*ld, caller's bus order, device FP64.  Asynchronous. */
hinv_status chol_solve(chol_handle h, const double* d_b, double* d_x, int32_t nrhs, int32_t ld, void* stream);
hinv_status chol_get_info(chol_handle h, chol_info_t* out);
hinv_status chol_destroy(chol_handle h);

/* ---- EMT time stepping (Section II, Eq. (1)) ---------------------------- */

/* Network: branch e is a series R[e]-L[e] between buses from[e] and to[e];
 * bus a has a shunt capacitance C[a] to ground; n_src current sources
 * amp*sin(2*pi*freq*t + phase) inject into src_bus.  Trapezoidal companion
 * models with step dt.  Host memory. */
typedef struct {
    int32_t n_bus, n_branch;
    const int32_t* from;
    const int32_t* to;
    const double* R;
    const double* L;
    const double* C;
    double dt;
    int32_t n_src;
    const int32_t* src_bus;
    const double* amp;
    const double* phase;
    double freq;
} emt_network;

/* Line-loss schedule for n_cases cases sharing one network: case k loses
 * branches loss_branch[loss_ptr[k] .. loss_ptr[k+1]) from steps
 * loss_step[...] on (step >= 1).  A lost branch carries no current from that
 * step on (it is removed from G and its history is dropped).  NULL pointers
 * with n_cases >= 1 mean no scheduled losses.  Host memory. */
typedef struct {
    int32_t n_cases;
    const int32_t* loss_ptr;     /* [n_cases+1] */
    const int32_t* loss_step;    /* [loss_ptr[n_cases]] */
    const int32_t* loss_branch;  /* [loss_ptr[n_cases]] */
} emt_cases;

/* The network's nodal conductance matrix G (trapezoidal companions:
 * g = 1/(R + 2L/dt) per branch, 2C/dt per shunt; Section II) as the full
 * symmetric CSR that hinv_build takes, in the network's bus order.  Call with
 * row_ptr == NULL to get *nnz only; otherwise row_ptr [n_bus+1], col_idx and
 * val [*nnz] (host memory, caller-owned) are filled. */
hinv_status emt_network_csr(const emt_network* net, int32_t* row_ptr, int32_t* col_idx, double* val, int64_t* nnz);

/* The three-phase G of the same network (Section III.A: each bus has three
 * phases): rows 3a + p, p = 0..2; branch e is a three-phase series R-L with
 * self inductance L[e] and mutual inductance mutual * L[e] between any two
 * phases, so its companion is the 3x3 admittance (R I + (2/dt) L_e)^{-1};
 * shunt 2C/dt on each phase.  0 <= mutual < 0.5 (SPD), else HINV_E_INVALID.
 * row_ptr [3 n_bus + 1]; otherwise as emt_network_csr.  For hinv_build, a
 * three-phase tree maps all three rows of a bus to the bus's leaf (a leaf then
 * holds at most HINV_MAX_LEAF / 3 buses).  emt3_create runs the EMT time loop
 * on this G. */
hinv_status emt_network3_csr(const emt_network* net, double mutual, int32_t* row_ptr, int32_t* col_idx,
                             double* val, int64_t* nnz);

/* Three-phase EMT time loop (Section II, Eq. (1), on the three-phase network
 * of Section III.A): G is emt_network3_csr's, rows 3a + p of bus a's phases
 * p = 0..2 in every vector and record.  Line e's trapezoidal companion is the
 * 3x3 admittance Y = (R I + (2/dt) L_e)^{-1}, L_e = L[e]((1 - mutual) I +
 * mutual J): its phase currents are i^n = Y v_ft^n + h^n with the history
 * h^{n+1} = Y v_ft^n + A i^n, A = Y ((2/dt) L_e - R I), v_ft the three phase
 * differences between its buses; shunt C[a] and its trapezoidal history per
 * phase.  Source q drives phase p of its bus with amp*sin(2 pi f t + phase +
 * shift[p]) (host [3]; NULL: 0, -2pi/3, +2pi/3, a balanced set).  tree is the
 * network's bus-level tree; each leaf then owns 3x its buses as rows (at most
 * HINV_MAX_LEAF).  loss_branch of the cases names lines: a lost line loses its
 * three phases, held as three changes w_p = e_from,p - e_to,p coupled by D =
 * -Y (G <- G + W D W^T, the capacitance then takes D^{-1} = -Z), so a case
 * holds at most max_mod_rank / 3 line losses (RANK_LIMIT beyond).  Engines:
 * one workgroup per case (kernel_mode 2, and the automatic choice when the
 * case fits its LDS in FP64 or FP32 storage) or one launch per phase
 * (kernel_mode 1, any storage precision); other modes HINV_E_INVALID.  The handle takes
 * emt_step, emt_lose_line (line index), emt_sync_status, emt_get_step,
 * emt_get_stats and emt_destroy as a single-phase one does; emt_update_line
 * and serve_attach refuse it with HINV_E_INVALID.  Other errors as
 * emt_workspace_size / emt_create, plus HINV_E_INVALID for mutual outside
 * [0, 0.5) or a non-finite shift. */
hinv_status emt3_workspace_size(const emt_network* net, double mutual, const double* shift, const hinv_tree* tree,
                                const hinv_options* opt, const emt_cases* cases, size_t* bytes);
hinv_status emt3_create(const emt_network* net, double mutual, const double* shift, const hinv_tree* tree,
                        const hinv_options* opt, const emt_cases* cases, void* d_ws, size_t ws_bytes, void* stream,
                        emt_handle* out);

hinv_status emt_workspace_size(const emt_network* net, const hinv_tree* tree, const hinv_options* opt,
                               const emt_cases* cases, size_t* bytes);

/* Build the hierarchical inverse of the network's G, the SMW factors of every
 * scheduled loss, and the initial state (v = 0, branch currents 0, capacitor
 * currents consistent with KCL at t = 0).  The next step is step 1.
 * Synchronises the stream. */
hinv_status emt_create(const emt_network* net, const hinv_tree* tree, const hinv_options* opt,
                       const emt_cases* cases, void* d_ws, size_t ws_bytes, void* stream, emt_handle* out);

/* Advance every case by n_steps steps: at step n, solve G_n v_n = i_in(t_n) + i_his
 * (t_n = n*dt) and update the trapezoidal history currents.  If d_v_record
 * is not NULL, v of case k at the j-th step of this call (bus order of the
 * network) is written to d_v_record[(j*n_cases + k)*n_bus + a]; d_b_record
 * likewise receives the right-hand side.  Asynchronous on the stream. */
hinv_status emt_step(emt_handle c, int32_t n_steps, double* d_v_record, double* d_b_record, void* stream);

/* Lose branch `branch` of case `case_idx` from the next step on (Algorithm 2's
 * situation, handled by a rank-1 SMW correction).  Synchronises the stream. */
hinv_status emt_lose_line(emt_handle c, int32_t case_idx, int32_t branch, void* stream);

/* Change the network of every case from the next step on by a memoryless
 * conductance delta_g between buses a and b (b = -1: between a and ground),
 * G <- G + delta_g (e_a - e_b)(e_a - e_b)^T: a fault switched on (delta_g =
 * 1/R_fault) or off again (its negative), the scenario of Section V.C.  The
 * stored inverse is rebuilt locally as by hinv_update_line (Section IV,
 * Algorithm 2 made exact: the result equals a fresh build of the new G), then
 * each case's line losses are re-applied to the new base and the engine's
 * per-workgroup tables take G's new values.  The element carries no history
 * current, so the state of the time loop is kept as it is.  Same argument
 * rules and errors as hinv_update_line (a and b in the network's bus order);
 * if the change, or a case's losses on top of it, makes G indefinite or
 * singular, nothing changes and HINV_E_NOT_SPD / HINV_E_SINGULAR is returned.
 * `out` (may be NULL) receives what was rebuilt.  Synchronises the stream. */
hinv_status emt_update_line(emt_handle c, int32_t a, int32_t b, double delta_g, void* stream,
                            hinv_update_info* out);

/* Device-side status of the steps run since the last call (call after the
 * stream is idle; clears it).  HINV_E_NO_CONVERGENCE: in mixed precision a
 * step's last correction ||dv||/||v|| exceeded rel_tol; HINV_E_NOT_SPD: a
 * non-finite value; HINV_E_DEVICE: a cooperative engine's inter-workgroup
 * barrier timed out or a line change's endpoint had no row in a workgroup's
 * tables (the trajectory is then invalid). */
hinv_status emt_sync_status(emt_handle c);

/* Index of the next step to be computed (1 after emt_create). */
hinv_status emt_get_step(emt_handle c, int64_t* step);

/* Checkpoint and resume of the time loop (Eq. (1)-(2): the state that carries
 * one step into the next).  A state holds the next step's index, every case's
 * right-hand side b, voltages v (the warm start of the refined paths),
 * capacitor histories (rows in the network's bus order) and branch histories
 * (the network's branch order), every case's line losses (step, branch:
 * scheduled, past and dynamic ones alike) and the base-matrix changes made by
 * emt_update_line since emt_create, with a fingerprint of the network.
 * emt_state_size: bytes of the handle's current state (host only).
 * emt_save_state: synchronises the stream, then copies the state into `buf`
 * (host memory, caller-owned, >= emt_state_size bytes).
 * emt_load_state: resumes a handle created on the same network (any tree,
 * engine or precision) from a state: the handle's base-matrix changes must be
 * the first ones of the state's (the rest are applied with emt_update_line),
 * its cases take the state's line losses and vectors, and its next step is
 * the state's.  With the same tree, engine and precision the resumed run
 * equals the uninterrupted one bitwise.  HINV_E_INVALID for a buffer that is
 * too short or not a state of this library, another network, case count or
 * phase count, or diverging base-matrix changes; HINV_E_RANK_LIMIT when a
 * case has more losses than the handle's max_mod_rank holds; the handle is
 * unchanged after these.  Errors while applying the state (HINV_E_NOT_SPD,
 * HINV_E_DEVICE) can leave it partly loaded.  Synchronises the stream. */
hinv_status emt_state_size(emt_handle c, size_t* bytes);
hinv_status emt_save_state(emt_handle c, void* buf, size_t bytes, void* stream);
hinv_status emt_load_state(emt_handle c, const void* buf, size_t bytes, void* stream);

/* Refinement statistics since emt_create (mixed precision): total applies,
 * largest final ||dv||/||v|| seen.  Synchronises nothing; call after the
 * stream is idle. */
hinv_status emt_get_stats(emt_handle c, int64_t* applies, double* max_rel_update);

/* Per-step timing for latency percentiles: while set, every fused emt_step
 * launch writes the GPU wall clock (wall_clock64(), constant rate, see
 * hipDeviceAttributeWallClockRate) after each step of case 0 into
 * d_clock[j], j = 0 .. min(n_steps, capacity)-1 of that call (device memory,
 * caller-owned).  d_clock == NULL switches it off.  The per-kernel engine
 * does not write it. */
hinv_status emt_set_step_clock(emt_handle c, int64_t* d_clock, int64_t capacity);

/* Rate of that wall clock on device `device`, in kHz. */
hinv_status hinv_wall_clock_khz(int32_t device, int32_t* khz);

hinv_status emt_destroy(emt_handle c);

/* ---- Serving: continuous batching of EMT cases -------------------------- */

/* A pool of single-case EMT handles advanced together: each serve_step is one
 * launch that advances every attached case by n_steps steps, one workgroup
 * per case, each case with its own network, hierarchy, line losses and state
 * (cases whose vectors do not fit a workgroup's LDS keep them in their own
 * workspace).  Cases can be attached and detached between steps, so requests
 * are admitted as slots free up.  A case's arithmetic does not depend on the
 * other cases in the launch.  The pool's precision and warm start must match
 * each attached case's options; refinement count and tolerance are the
 * case's own.  Do not call emt_step on an attached handle. */
typedef struct serve_ctx* serve_handle;

hinv_status serve_workspace_size(int32_t max_slots, size_t* bytes);
hinv_status serve_create(const hinv_options* opt, int32_t max_slots, void* d_ws, size_t ws_bytes, serve_handle* out);
/* d_v_record (optional, device): row j receives the case's v at its j-th step after attaching (bus order of
 * its network), j < record_capacity.  Synchronises the stream. */
hinv_status serve_attach(serve_handle s, emt_handle c, double* d_v_record, int64_t record_capacity, void* stream,
                         int32_t* slot_id);
/* Synchronises the stream, then removes the case from the pool. */
hinv_status serve_detach(serve_handle s, int32_t slot_id, void* stream);
hinv_status serve_step(serve_handle s, int32_t n_steps, void* stream);
hinv_status serve_active(serve_handle s, int32_t* n_active);
hinv_status serve_destroy(serve_handle s);

const char* hinv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
