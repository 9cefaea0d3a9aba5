/*
 * fdbem -- fast directional Burton-Miller boundary element mat-vec and solver
 * for AMD Instinct MI355X (gfx950).  Public C ABI.
 *
 * Method: Cao, Wen, Xiao, Liu, "A fast directional BEM for large-scale
 * acoustic problems based on the Burton-Miller formulation" (arXiv 1311.5202).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Complex vectors are arrays of interleaved FP64 pairs (re, im), i.e.
 *    C99 "double complex" / torch.complex128, length N, in the CALLER's node
 *    order.  Device pointers ("_dev") must point to memory on the current HIP
 *    device; host pointers are read during the call only.
 *  - The plan owns every device allocation it makes; the caller owns the
 *    input/output buffers.  Calls are ordered on the HIP stream passed in
 *    (NULL = the default stream) and do not synchronise unless stated.
 *  - Normals point INTO the body (out of the acoustic domain): the orientation
 *    under which the integral representation of section 2.1 carries +dG/dn_y.
 *  - alpha = i/k (section 2.1, eq. eq_bm).
 *  - Return value: FDA_OK (0) or a negative FDA_E* code; nothing is thrown
 *    across the ABI.  fda_last_error() returns a thread-local message for the
 *    last failing call on the calling thread.
 */
#ifndef FDBEM_H
#define FDBEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FDA_OK = 0,
    FDA_EINVAL = -1,        /* bad argument (sizes, k <= 0, eps outside (0,1), null pointer) */
    FDA_ENOMEM = -2,        /* host or device allocation failed */
    FDA_EHIP = -3,          /* a HIP runtime call failed */
    FDA_NOT_CONVERGED = -4, /* GMRES reached maxit; x holds the last iterate */
    FDA_NONFINITE = -5,     /* NaN/Inf in an input vector or in the Krylov recurrence */
    FDA_EBREAKDOWN = -6,    /* GMRES breakdown before the tolerance was met */
    FDA_ENOTSUP = -7        /* option combination not supported */
};

/* Operators applied by fda_matvec (section 2.2 eqs. eq_hmat, eq_gmat, kcorrection,
 * section 5.1 eq. eq_sum).  w_j are the quadrature weights of the geometry. */
enum {
    FDA_OP_RAW_H = 0,  /* p_i = sum_{j!=i} w_j [dG/dn_y + alpha d2G/dn_x dn_y](x_i,y_j) u_j */
    FDA_OP_RAW_G = 1,  /* p_i = sum_{j!=i} w_j [G + alpha dG/dn_x](x_i,y_j) u_j              */
    FDA_OP_RAW_T1 = 2, /* p_i = sum_{j!=i} w_j [G + alpha dG/dn_y](x_i,y_j) u_j (eq. eq_sum)  */
    FDA_OP_BM_H = 3,   /* (1/2) u_i + sum_j Hbar_ij u_j: the sound-hard Burton-Miller operator,
                          raw H sum plus the locally corrected near field (needs elements)   */
    FDA_OP_BM_G = 4    /* sum_j Gbar_ij q_j: corrected G sum (needs elements)                */
};

/* OR'ed into an operator code: evaluate the near-field point sum and the far
 * field (S2M .. L2T) in FP32 (differences of positions and the correction
 * SpMV stay FP64).  Needs a plan built with FDA_PREC_FP32 or FDA_PREC_BOTH;
 * on an FP32-only plan it is implied. */
#define FDA_OP_FP32 0x100

enum { FDA_PREC_FP64 = 0, FDA_PREC_FP32 = 1, FDA_PREC_BOTH = 2 };

/* Geometry: Nystrom nodes with normals and weights; optionally the curved
 * quadratic elements they come from (needed for the local corrections).
 * Element e holds 6 geometric nodes (corners 0,1,2 counter-clockwise seen
 * from the acoustic side, then mid-edge nodes of edges 01, 12, 20), 18
 * doubles, and owns nodes 6e..6e+5 in the order of bem_nystrom_nodes. */
typedef struct {
    int64_t n_nodes;
    const double *pts; /* n_nodes x 3 */
    const double *nrm; /* n_nodes x 3, unit, into the body */
    const double *w;   /* n_nodes */
    int64_t n_elem;    /* 0, or n_nodes / 6 */
    const double *elem;/* n_elem x 6 x 3, or NULL */
} fda_geometry;

typedef struct {
    double svd_eps;     /* truncation of the pseudo-inverses (eq. eq_invr); 0 -> eps for the
                           low-frequency templates and eps/3 for the high-frequency ones
                           (fitted on a skeleton of the region the field is evaluated in,
                           they err about three times the truncation between its points) */
    double lowrank_eps; /* truncation of the low-rank M2L factors (eq. eq_lrdk); 0 -> eps;
                           < 0: no low-rank factors (every M2L applies K~)               */
    int leaf_cap;       /* max points per octree leaf; 0 -> 64                            */
    int leaf_rule;      /* 0: leaves are low-frequency cubes (w < lambda)                  */
    double c_d;         /* high-frequency near-field constant (section 3.1.1); 0 -> 1/pi  */
    int far_field;      /* 1: fast directional far field; 0: all pairs summed directly    */
    int lf_grid;        /* points per edge of low-frequency surface grids; 0 -> from eps  */
    int precision;      /* FDA_PREC_FP64, FDA_PREC_FP32 or FDA_PREC_BOTH (see FDA_OP_FP32) */
    int corrections;    /* bit 0: corrected H table, bit 1: corrected G table (needs elements) */
    int verbose;
    int wedge_factor;   /* directional wedges: cells per cube-face edge = wedge_factor * w / lambda; 0 -> 2 */
    int m2l_tile;       /* translation schedule: 0 -> operator chunks whose per-pair results
                           are summed per output in a fixed order (deterministic, default),
                           1 -> operator chunks with atomic adds, > 1 -> workgroup M2L tiles
                           of that size, < 0 -> per-target GEMV */
    double p2p_threshold; /* a far pair whose point counts multiply to at most this is summed
                             directly instead of translated; 0 -> 400, < 0 -> never */
    double coupling;    /* Burton-Miller coupling alpha = i * coupling / k (section 2.1,
                           eq. eq_bm); 0 -> 1, the value the paper uses.  -1 gives the
                           conjugate coupling (see bm_solve). */
    int autotune;       /* 1 (default): at build, time 16 and 32 pairs per M2L, M2M and L2L
                           chunk of the workgroup kernel on the plan's own lists and keep the
                           faster per translation and level (fda_stats: m2l_/m2m_/l2l_autotune;
                           levels on the wavefront kernel are timed, not tuned); 0: 16 */
    int slab_mb;        /* scratch for per-pair translation results, MiB per slab; 0 -> 1024 */
    int hf_template;    /* high-frequency templates: 0 (default) one per wedge orbit, check
                           points on the region where the wedge's outgoing field is evaluated
                           (M2L target cubes, parent check points), equivalent points on the
                           cube's surface; 1: the earlier circular check cone and ball of
                           equivalent points rotated to each wedge (larger s)               */
    int original;       /* 1: the method the paper improves on (section 4, Table 1), for
                           comparison: translations act on the equivalent densities with
                           the uncompressed pseudo-inverses R+ and M2L matrices K (no
                           matrix reduction of section 4.1, no low-rank M2L of section
                           4.2); same results up to rounding, larger operators; 0 default */
    int serial_slabs;   /* 0 (default): two scratch slabs of slab_mb each; every translation
                           launch also sums the previous slab's per-pair results (same sums
                           in the same order); 1: one slab, chunks and sums in separate
                           launches                                                        */
    int chunk_kernel;   /* translation chunks of the default schedule: 0 (default) one
                           wavefront per chunk for every translation list (one kind and
                           level) whose operators all fit it (dense, or low-rank with rank
                           at most 32), the workgroup kernel for the
                           other lists; 1: the workgroup kernel everywhere.  Results of the
                           two kernels differ by rounding only; neither depends on slab_mb. */
} fda_opts;

typedef struct fda_plan fda_plan;

/* Fill *o with the defaults listed above. */
int fda_default_opts(fda_opts *o);

/* Nystrom discretisation (section 2.2): nodes, unit normals (into the body)
 * and weights of the six-point degree-4 Gauss rule on each curved quadratic
 * element.  All host arrays; pts/nrm are 6*n_elem x 3, w is 6*n_elem. */
int bem_nystrom_nodes(int64_t n_elem, const double *elem, double *pts, double *nrm, double *w);

/* Locally corrected near-field table of one operator (section 2.2, eqs.
 * near field, local correction, kcorrection), host only, caller node order:
 * CSR rows i with entries dw_ij = wbar_j(K; x_i) - [j != i] w_j K(x_i, y_j)
 * over the nodes j of the elements in the local region D_i of x_i (elements
 * whose distance to x_i is at most twice their longest side).  op is
 * FDA_OP_BM_H (K = dG/dn_y + alpha d2G/dn_x dn_y) or FDA_OP_BM_G
 * (K = G + alpha dG/dn_x), alpha = i coupling / k (coupling 0 -> 1).  Call with row_ptr = col = val = NULL to get
 * *nnz_out; then with row_ptr (n_nodes+1), col (nnz) and val (2*nnz doubles,
 * interleaved complex) to fill them.  Nodes must be those of
 * bem_nystrom_nodes for the same elements. */
int bem_near_correction(int64_t n_elem, const double *elem, const double *pts, const double *nrm, const double *w,
                        double k, int op, double coupling, int64_t *nnz_out, int64_t *row_ptr, int64_t *col,
                        double *val);

/* Build a plan on the current HIP device: octree and lists (section 3.1.1),
 * point templates (section 3.1.2), their pseudo-inverses (section 4.1, eqs.
 * eq_svdr/eq_invr),
 * compressed translation operators (section 4.1, eqs. eq_cmps..eq_cmpt),
 * low-rank M2L factors (eq. eq_lrdk) and, with elements, the locally
 * corrected near field (section 2.2).  k > 0 is the wavenumber, eps in
 * (0,1) the controlling accuracy.  opts may be NULL (defaults).  Host work
 * is FP64; everything the mat-vec reads is uploaded.  Synchronous. */
int fda_build(const fda_geometry *geom, double k, double eps, const fda_opts *opts, fda_plan **out);

/* The host part of fda_build without a device: octree and lists (section
 * 3.1.1), templates (section 3.1.2, eqs. eq_svdr/eq_invr) and compressed
 * operators (sections 4.1, 4.2), described as the JSON of fda_stats (levels,
 * reduced dimensions s, pair and operator counts, work per phase).  For
 * inspecting and sizing a plan on a machine without a GPU.  Writes at most
 * len bytes including the terminating zero (FDA_EINVAL if it does not fit). */
int fda_analyze(const fda_geometry *geom, double k, double eps, const fda_opts *opts, char *json_buf, size_t len);

/* out_dev = Op(in_dev) for op in FDA_OP_*: both complex128[N] device
 * buffers in caller order (they must not overlap).  BM_* ops need a plan
 * built with elements.  Stream-ordered, no synchronisation. */
int fda_matvec(fda_plan *plan, int op, const void *in_dev, void *out_dev, void *hip_stream);

/* fda_matvec that allocates nothing, for callers that cannot allocate
 * device memory during the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same operators, arguments and
 * result as fda_matvec (never through a captured graph).  The per-pair
 * translation results that fda_matvec keeps in the plan's slab buffer go to
 * a static 256 MiB device array of the library instead; each device holds
 * its own copy until the process ends, and every call on that device shares
 * it, so calls that overlap on one device race (order them on one stream).
 * FDA_EINVAL if the plan's largest slab needs more than 256 MiB (build it
 * with slab_mb <= 256), if it uses a schedule other than the operator
 * chunks (m2l_tile 0 or 1), or if the plan's device is not current. */
int fda_matvec_noalloc(fda_plan *plan, int op, const void *in_dev, void *out_dev, void *hip_stream);

/* Solve Op x = rhs by GMRES (section 2.2 eq. Axb; right preconditioned,
 * x0 = 0, restart length `restart`, Arnoldi by classical Gram-Schmidt with
 * re-orthogonalisation, FP64).  Stops when ||b - A x|| / ||b|| <= tol.
 * rhs_dev/x_dev: complex128[N] device buffers.  iters_out, relres_out may be
 * NULL; resid_hist (host, maxit+1 doubles) may be NULL.  precond: 0 none,
 * 1 block-Jacobi on the corrected near-field leaf blocks, 2 block-Jacobi plus
 * the learned coupling loaded by fda_net_attach, 3 the restricted additive
 * Schwarz rows R_b that the coupling is trained towards (see fda_net_*).  Synchronises the
 * stream once per iteration.  FDA_NOT_CONVERGED leaves the last iterate. */
int bm_solve(fda_plan *plan, int op, const void *rhs_dev, double tol, int maxit, int restart, int precond,
             void *x_dev, int *iters_out, double *relres_out, double *resid_hist, void *hip_stream);

/* Right-hand side of the sound-hard problem (section 5.3): incident plane
 * wave u_inc = exp(i k x.d) with unit direction d[3];
 * b_i = u_inc(x_i) + alpha du_inc/dn_x(x_i).  rhs_dev: complex128[N]. */
int fda_rhs_plane_wave(fda_plan *plan, const double d[3], void *rhs_dev, void *hip_stream);

/* Right-hand side of a Neumann problem without incident wave, e.g. the
 * radiation of a vibrating body (section 2.1, eq. eq_bm with u_inc = 0;
 * section 5.2): rhs = (S + alpha M) q - alpha c q with c = 1/2, where the
 * layer operators carry the local corrections (the FDA_OP_BM_G operator of
 * this plan) and alpha = i coupling / k.  q_dev: the normal derivative
 * du/dn (normal into the body), rhs_dev: output; both complex128[N] device
 * buffers in caller order that must not overlap.  Needs a plan built with
 * elements and corrections & 2 (FDA_EINVAL otherwise).  Solve with
 * bm_solve(FDA_OP_BM_H, rhs) for u on the surface.  Stream-ordered. */
int fda_rhs_neumann(fda_plan *plan, const void *q_dev, void *rhs_dev, void *hip_stream);

/* JSON description of the plan (levels, slot counts, ranks, memory, set-up
 * and per-phase timings of the last timed mat-vec).  Writes at most len bytes
 * including the terminating zero; returns FDA_EINVAL if it does not fit. */
int fda_stats(const fda_plan *plan, char *json_buf, size_t len);

/* Enable (1) or disable (0) per-phase HIP-event timing of fda_matvec.  Events
 * are recorded on the mat-vec's stream without synchronising. */
int fda_set_timing(fda_plan *plan, int on);

/* Per-phase times (milliseconds), averaged over the timed mat-vecs since the
 * previous call (at most the last 64), in the order P2P, S2M, M2M, M2L, L2L,
 * L2T, near correction, permutations; n: capacity of ms.  Waits for the
 * recorded events, then starts a new averaging window. */
int fda_phase_times(fda_plan *plan, double *ms, int n);

/* ---- captured mat-vecs and batches of plans ----------------------------
 * Not steps of the paper's method: ways of launching it.  With graphs on, a
 * plan captures each (operator, input, output) mat-vec of fda_matvec and of
 * bm_solve into a HIP graph the first time and replays it afterwards
 * (bm_solve steps use fixed internal buffers, so one graph serves a whole
 * solve); at most 8 graphs are kept per plan (fda_stats: graphs_captured),
 * and turning graphs off releases them.  Results are bitwise those of the
 * eager launches.  Graphs are bypassed while fda_set_timing is on. */
int fda_set_graph(fda_plan *plan, int on);

/* A batch groups plans on the current device (each plan at most once; the
 * plans must outlive the batch).  fda_batch_matvec applies op to every
 * instance, in_dev[i] -> out_dev[i] (device complex128 vectors of plan i's
 * length), as ONE graph launch in which the instances run concurrently on 16
 * forked streams; the graph is re-captured when op or a pointer changes.
 * fda_batch_solve runs bm_solve for every instance (op, tol, maxit, restart,
 * precond as in bm_solve) from a pool of host threads, one stream each, with
 * graphs on; per-instance iterations, relative residuals and status codes go
 * to the host arrays iters, relres (may be NULL) and status.  Returns
 * FDA_NOT_CONVERGED if any instance did not converge.  Synchronous. */
typedef struct fda_batch fda_batch;
int fda_batch_create(fda_plan *const *plans, int n, fda_batch **out);
int fda_batch_matvec(fda_batch *b, int op, const void *const *in_dev, void *const *out_dev, void *hip_stream);
int fda_batch_solve(fda_batch *b, int op, const void *const *rhs_dev, double tol, int maxit, int restart,
                    int precond, void *const *x_dev, int *iters, double *relres, int *status);
void fda_batch_destroy(fda_batch *b);

/* ---- learned coupling correction of the block-Jacobi preconditioner ----
 * Not part of the paper's method: a preconditioner for bm_solve.  Blocks b
 * are the octree leaves cut into pieces of at most 64 points; E_b is the block
 * followed by up to 64 of its nearest points among the leaf's direct-sum
 * sources (ne_b <= 128).  With precond = 2 bm_solve applies
 *   z_b = A_bb^{-1} v_b + U_b (W_b^H v_{E_b}),
 * A_bb the corrected near-field block of BM_H, U_b (n_b x 4) and W_b
 * (ne_b x 4) produced row by row by a small network (12 features of the pair
 * (b, j) -> 32 tanh -> 16 outputs: Re/Im of row j of U, then of W).
 * Training target: the restricted additive Schwarz rows R_b =
 * [(A|E_b)^{-1}]_{b,E_b}; loss = sum_b c_b w_b ||[A_bb^{-1} 0] + U_b W_b^H -
 * R_b||_F^2 with w_b = 1/||R_b - [A_bb^{-1} 0]||_F^2 (0 when that is at most
 * 1e-12 ||R_b||_F^2) and c_b = 1 unless set from the method's own GMRES run
 * by fda_net_weight_blocks.  Features, forward, backward and Adam run on the GPU;
 * the network lives on the device current at fda_net_create.  Every call is
 * synchronous. */
typedef struct fda_net fda_net;

int fda_net_num_params(void);
int fda_net_create(uint64_t seed, fda_net **out);
void fda_net_destroy(fda_net *net);
/* parameters: host arrays of fda_net_num_params() doubles, laid out as W1
 * (32 x 12 row-major), b1 (32), W2 (16 x 32 row-major), b2 (16) */
int fda_net_get_params(const fda_net *net, double *params);
int fda_net_set_params(fda_net *net, const double *params);  /* FDA_EINVAL on non-finite values */
/* loss and gradient (host array, may be NULL) over the plan's blocks.  Builds
 * the plan's overlapping sets and targets on first use (the plan needs
 * elements: FDA_EINVAL otherwise) and unloads factors loaded by
 * fda_net_attach (load them again before precond = 2). */
int fda_net_loss_grad(fda_net *net, fda_plan *plan, double *loss, double *grad);
/* one Adam step (beta 0.9, 0.999) of learning rate lr > 0 on the plan's
 * blocks; *loss (may be NULL) is the loss before the step */
int fda_net_train_step(fda_net *net, fda_plan *plan, double lr, double *loss);
/* block weights c_b of the plan's training loss from the method's own GMRES
 * run: `iters` steps of the block-Jacobi preconditioned solve of FDA_OP_BM_H
 * with right-hand side rhs_dev (complex128[N] on the device), then c_b = the
 * energy of its Krylov vectors (the directions its residuals take) on block
 * b's overlapping set E_b, scaled to mean 1; iters = 0 restores c_b = 1.
 * Needs a plan built with elements (FDA_EINVAL otherwise). */
int fda_net_weight_blocks(fda_plan *plan, const void *rhs_dev, int iters);
/* evaluate the network on the plan and load the factors for precond = 2;
 * net = NULL unloads them (precond = 2 then reports FDA_ENOTSUP) */
int fda_net_attach(fda_net *net, fda_plan *plan);
/* loss and gradient for caller data, all device pointers: per block b,
 * feature rows [pair_off[b], pair_off[b] + block_ne[b]) of the n_rows x 12
 * array (block points first), the inverse block at inv_off[b] (n_b x n_b),
 * the target at target_off[b] (n_b x ne_b), column-major complex128, and the
 * block weights c_b (n_blocks doubles, may be NULL for c_b = 1).
 * FDA_EINVAL unless 1 <= n_b <= 64, n_b <= ne_b <= 128 and the rows lie in
 * the array; the complex arrays must hold the blocks at their offsets.  For
 * checking the kernels against an independent implementation. */
int fda_net_loss_grad_raw(fda_net *net, int n_blocks, const int64_t *pair_off, const int *block_n,
                          const int *block_ne, const int64_t *inv_off, const int64_t *target_off, int64_t n_rows,
                          const double *features, const void *block_inv, const void *targets,
                          const double *block_weight, double *loss, double *grad);

/* Release every device and host resource of the plan (NULL is allowed). */
void fda_destroy(fda_plan *plan);

/* Message of the last non-zero status on this thread ("" if none). */
const char *fda_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FDBEM_H */
