/*
 * pseudoflow.h -- C ABI of the MI355X (gfx950) pseudo-flow continuous max-flow
 * solvers: entropic Bregman proximal label steps and Chambolle flow steps for
 * the Potts, hierarchical (HMF) and DAG (DAGMF) models, and the Ishikawa chain
 * (Baxter, Rajchl, Yuan, Peters, "A Proximal Bregman Projection Approach to
 * Continuous Max-Flow Problems Using Entropic Distances").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid.     A batch of B independent problems on a Z x Y x X grid (2-D problems
 *           have ndim == 2 and nz == 1).  Unit spacing; forward differences
 *           with a zero gradient on the last index of each axis; the
 *           divergence is the negative adjoint of that gradient.
 * Layout.   Every field is a dense float array [B][F][Z][Y][X], x fastest.
 *           Flows are [B][n_node][ndim][Z][Y][X], component k = axis x, y, z
 *           for k = 0, 1, 2.
 * Labels.   D holds one data term per end-label (leaf), leaves numbered in
 *           ascending node id.  Internal labels carry no data term.
 * Graphs.   Node 0 is the source.  Edge weights default to 1/|parents(child)|
 *           and the weighted path sums from the source to every leaf must be 1.
 * Memory.   Every device pointer is allocated and freed by the caller.  The
 *           library never allocates device memory: the solver state lives in
 *           the caller's workspace (pf_workspace_bytes), which also carries it
 *           from one call to the next (warm_start).  Host arrays are read
 *           during the call only.
 * Streams.  Work is enqueued on `stream` (a hipStream_t; NULL is the default
 *           stream).  The call returns without synchronising unless it must
 *           read results back: gap_every > 0, final_energy, check_inputs or
 *           timing_stride > 0.  Then it synchronises `stream` before returning.
 * Errors.   The return value is a pf_status; pf_last_error() gives a message
 *           (thread-local, valid until the next call on the thread).  Every
 *           argument and graph check happens before the first launch and an
 *           invalid call leaves all outputs untouched.  PF_EHIP reports a HIP
 *           runtime failure and PF_ENONFINITE a NaN/Inf found by check_inputs
 *           or by a gap evaluation; after those two, outputs are undefined.
 */
#ifndef PSEUDOFLOW_H
#define PSEUDOFLOW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PF_ABI_VERSION 3      /* 3: PF_KERNEL_LDS */
#define PF_MAX_LEAVES 16     /* end-labels per problem */
#define PF_MAX_NODES 32      /* non-source nodes per problem */
#define PF_STATIC_SCRATCH_BYTES (128u << 20)   /* device scratch of solve_dagmf_static */

typedef enum {
    PF_OK = 0,
    PF_EINVAL = -1,          /* bad argument (null/misaligned pointer, size, c, tau, ...) */
    PF_EGRAPH = -2,          /* label graph rejected (cycle, orphan, weights, not a tree) */
    PF_ENOMEM = -3,          /* workspace smaller than pf_workspace_bytes() */
    PF_EHIP = -4,            /* HIP runtime error */
    PF_ENONFINITE = -5,      /* NaN/Inf in the inputs or in a gap evaluation */
    PF_EUNSUPPORTED = -6     /* valid but outside this build (too many labels, ...) */
} pf_status;

typedef enum { PF_FP32 = 0, PF_BF16 = 1, PF_FP16 = 2 } pf_storage;

typedef enum {
    PF_S_NODE_SCALAR = 0,    /* S: HOST float[n_node], one constant per flow */
    PF_S_SHARED_FIELD = 1,   /* S: device float[B][Z][Y][X], shared by every flow */
    PF_S_NODE_FIELD = 2      /* S: device float[B][n_node][Z][Y][X] */
} pf_s_mode;

typedef enum {
    PF_KERNEL_AUTO = 0,      /* the faster variant as measured on MI355X: LDS for
                                batches of 8 or more 2-D problems that fit whole,
                                and for other 2-D problems of at most 8 leaves and
                                8 flows up to 2^21 voxel-fields (voxels x problems
                                x (n_leaf + n_node)); for 3-D Potts FUSED2 up to 8
                                labels (every storage type), beyond that FUSED with
                                fp32 state; FUSED for 3-D label graphs (DAGMF, HMF)
                                of at most 16 flows and 16 leaves with fp32 state,
                                and in every storage type for 3-D graphs whose
                                end-labels are the last nodes, under 4 internal
                                nodes with 4, 8, 12 or 16 leaves, under 8 with 8 or
                                12, or under 3 with 8; FUSED for the 3-D Ishikawa
                                chain with fp32 state unless it has 5, 9 or 13
                                labels, and with 16-bit state up to 4 labels;
                                two-pass otherwise */
    PF_KERNEL_TWO_PASS = 1,  /* label pass then flow pass, state updated in place */
    PF_KERNEL_FUSED = 2,     /* one pass per iteration, state ping-ponged (at most 16
                                leaves and 16 flows; 3-D label graphs run the flow
                                step of one iteration and the label step of the next
                                in one pass, entered and left with a label pass and a
                                flow pass around every gap check; not for the
                                Ishikawa chain in 2-D); the same result as
                                PF_KERNEL_TWO_PASS bit for bit */
    PF_KERNEL_FUSED2 = 3,    /* one pass per two iterations (3-D Potts, n_leaf <= 8;
                                PF_EUNSUPPORTED otherwise), state ping-ponged; an
                                iteration that ends on a gap check, or the last of an
                                odd count, runs the one-iteration pass */
    PF_KERNEL_LDS = 4        /* 2-D problems of at most 8 leaves and 16 flows
                                (PF_EUNSUPPORTED otherwise), iterations in LDS: for
                                batches of 8 or more problems of at most 4096 voxels
                                whose float32 state, n_leaf + 2 n_node floats per
                                voxel, fits in 160 KB, one block per problem and one
                                launch for every iteration up to the next gap check
                                (state in place); otherwise tiles with ghost zones 8
                                voxels wide, one block per tile and up to 8
                                iterations per launch (state ping-ponged); the same
                                result as PF_KERNEL_TWO_PASS bit for bit */
} pf_kernel;

typedef struct {
    int32_t batch, ndim, nz, ny, nx;
} pf_grid;

typedef struct {
    int32_t n_nodes;         /* including the source (node 0) */
    int32_t n_edges;
    const int32_t *parent;   /* host [n_edges] */
    const int32_t *child;    /* host [n_edges] */
    const double *weight;    /* host [n_edges], or NULL for 1/|parents(child)| */
} pf_graph;

typedef struct {
    int32_t iters;           /* iterations to run, >= 0 */
    float c;                 /* entropic proximal weight, > 0 */
    float tau;               /* flow step parameter, > 0 (the step is c*tau) */
    int32_t storage;         /* pf_storage of the label and flow state */
    int32_t kernel;          /* pf_kernel */
    int32_t warm_start;      /* 1: continue from the state in the workspace */
    int32_t gap_every;       /* > 0: evaluate energy/dual every gap_every iterations */
    double gap_tol;          /* > 0: stop once (E - P) <= gap_tol * |E| at an evaluation */
    int32_t final_energy;    /* 1: evaluate energy, dual and gap after the last iteration */
    int32_t check_inputs;    /* 1: reject NaN/Inf in D and NaN/Inf/negative S first */
    int32_t timing_stride;   /* > 0: time the launch starting every timing_stride-th
                                iteration with HIP events (one launch covers two
                                iterations with PF_KERNEL_FUSED2; with PF_KERNEL_LDS
                                the launches of every chunk of iterations up to the
                                next gap check are timed as one) */
    void *workspace;         /* device, 256-byte aligned, caller-owned */
    size_t workspace_bytes;
    /* Differentiable solves (float32 state only).  With tape != NULL the
     * forward solve records the state before every ckpt_every-th iteration
     * (pf_tape_bytes) for the *_backward entry points; it then runs the
     * two-pass kernels and needs gap_tol == 0 and warm_start == 0. */
    int32_t ckpt_every;      /* >= 1 when tape != NULL */
    void *tape;              /* device, 256-byte aligned, caller-owned, or NULL */
    size_t tape_bytes;
} pf_params;

typedef struct {
    float *u;                /* device out [B][n_leaf][Z][Y][X] fp32, or NULL */
    int32_t *labels;         /* device out [B][Z][Y][X] argmax leaf (ties: lowest), or NULL */
    float *q;                /* device out [B][n_node][ndim][Z][Y][X] fp32, or NULL */
    float *ell;              /* device out [B][n_leaf][Z][Y][X] fp32 log-labels ln u, or NULL */
    double *gap_history;     /* host out [gap_history_cap] absolute gaps, or NULL */
    int32_t gap_history_cap;
    /* filled by the call */
    int32_t gap_history_len;
    int32_t iters_done;
    double energy;           /* primal energy E(u), summed over the batch (fp64) */
    double dual;             /* pseudo-flow dual P(q), summed over the batch (fp64) */
    double gap;              /* E - P */
    double max_simplex_err;  /* max over voxels of |sum_L u_L - 1| */
    double max_flow_excess;  /* max over flows and voxels of |q_A| - S_A (<= 0 if feasible) */
    double kernel_ms;        /* summed duration of the timed launches */
    int32_t kernel_timed;    /* number of iterations those launches covered */
} pf_result;

/* Bytes of device workspace needed for a problem.  n_leaf end-labels and
 * n_node non-source nodes carrying a flow (Potts: both equal the label count;
 * Ishikawa with N+1 labels: n_leaf = N+1, n_node = N).  `params` selects the
 * storage type and kernel; only those two fields are read.  Returns 0 for
 * arguments no solver accepts. */
size_t pf_workspace_bytes(const pf_grid *grid, int32_t n_leaf, int32_t n_node,
                          const pf_params *params);

/* The kernel PF_KERNEL_AUTO runs for an unrecorded solve of this problem:
 * identity != 0 for the Potts model, 0 for a label graph (DAGMF, HMF, and the
 * Ishikawa chain, whose AUTO follows the same rule and which is told from the
 * others by having fewer flows than labels, n_node = n_leaf - 1; a graph is
 * taken to number its end-labels last, as every graph whose leaves have the
 * highest node ids does); storage is a pf_storage.  Host only, no device work.  Returns PF_KERNEL_TWO_PASS, PF_KERNEL_FUSED,
 * PF_KERNEL_FUSED2 or PF_KERNEL_LDS, or -1 for arguments no solver accepts. */
int32_t pf_auto_kernel(const pf_grid *grid, int32_t n_leaf, int32_t n_node, int32_t identity,
                       int32_t storage);

/* Pseudo-flow Potts model (Algorithm 1, Potts section: relaxed Potts energy,
 * pseudo-flow dual max_{|q_L|<=S_L} sum_x min_L (D_L + div q_L), closed-form
 * entropic label update and the Chambolle flow update).  One iteration is
 *   d_L  = D_L + div q_L
 *   u_L <- u_L exp(-d_L/c) / sum_L' u_L' exp(-d_L'/c)   (max-subtracted log-sum-exp)
 *   q_L <- Proj_{|q_L| <= S_L}(q_L - c tau grad u_L)
 * starting from u = 1/n_labels, q = 0.  D: device float[B][n_labels][Z][Y][X].
 * S: per s_mode with n_node = n_labels. */
int solve_potts(const pf_grid *grid, int32_t n_labels, const float *D, const float *S,
                int32_t s_mode, const pf_params *params, pf_result *result, void *stream);

/* Pseudo-flow DAGMF model (Algorithm 2, DAGMF section): top-down flow excess
 *   d_A = div q_A + sum_{P in parents(A), P != source} w_(P,A) d_P  (+ D_A at leaves),
 * the entropic label update over the end-labels, and bottom-up implicit labels
 *   U_A = sum_{C in children(A)} w_(A,C) U_C  (U = u at leaves)
 * driving q_A <- Proj_{|q_A| <= S_A}(q_A - c tau grad U_A) for every non-source
 * node A.  D: device float[B][n_leaf][Z][Y][X]; S per s_mode with n_node =
 * n_nodes - 1, flow A-1 belonging to node A. */
int solve_dagmf(const pf_grid *grid, const pf_graph *graph, const float *D, const float *S,
                int32_t s_mode, const pf_params *params, pf_result *result, void *stream);

/* Hierarchical max-flow: solve_dagmf restricted to trees (every non-source
 * node has exactly one parent, unit weights), the HMF special case of the
 * DAGMF section.  A graph that is not such a tree returns PF_EGRAPH. */
int solve_hmf(const pf_grid *grid, const pf_graph *graph, const float *D, const float *S,
              int32_t s_mode, const pf_params *params, pf_result *result, void *stream);

/* Pseudo-flow Ishikawa chain (Algorithm 3): labels L_0..L_N (n_labels = N+1),
 * flows q_1..q_N; flow excess d_i = D_i + sum_{j<=i} div q_j and the flow of
 * L_i driven by U_i = sum_{j>=i} u_j.  D: device float[B][N+1][Z][Y][X];
 * S per s_mode with n_node = N.  Supports PF_KERNEL_TWO_PASS, PF_KERNEL_LDS,
 * PF_KERNEL_FUSED on 3-D grids, and AUTO (the rule of pf_auto_kernel with
 * identity = 0: LDS for small 2-D problems, FUSED on 3-D grids where it
 * measured faster, else two-pass). */
int solve_ishikawa(const pf_grid *grid, int32_t n_labels, const float *D, const float *S,
                   int32_t s_mode, const pf_params *params, pf_result *result, void *stream);

/* solve_dagmf without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  The arguments and results are those of
 * solve_dagmf, except that params->workspace must be NULL and
 * params->workspace_bytes 0 (else PF_EINVAL), params->tape NULL and
 * params->timing_stride 0 (else PF_EUNSUPPORTED: no tape, no HIP events).  The
 * solver state lives in a static device array of PF_STATIC_SCRATCH_BYTES
 * (128 MiB) that every GPU the library runs on holds until the process ends;
 * a problem whose state and buffers need more (the workspace layout of the
 * kernel the call runs) returns PF_ENOMEM before any device work.  Under
 * PF_KERNEL_AUTO the call takes the two-pass kernels (one copy of the state)
 * where the faster kernel's layout (two copies) would not fit.  The call allocates nothing: no hipMalloc, no
 * hipFree, no HIP events.  It runs on the current device, and a non-NULL
 * stream must belong to it (else PF_EINVAL).  Every call on a GPU shares that
 * GPU's array and it keeps the last call's contents: the solver initialises
 * the state it needs (warm_start = 1 continues from whatever the last call on
 * that GPU left, meaningful only for the same problem), and calls that
 * overlap on one GPU (other streams, other host threads) race on it. */
int solve_dagmf_static(const pf_grid *grid, const pf_graph *graph, const float *D,
                       const float *S, int32_t s_mode, const pf_params *params,
                       pf_result *result, void *stream);

/* Full-flow counterpart of solve_potts, kept to measure what the pseudo-flow
 * representation saves (Potts primal max-flow and primal-dual models, section
 * "Pseudo-Flow Approach to the Potts Model"; the paper names the full-flow
 * method but prints no algorithm for it).  Every variable of the primal-dual
 * model is explicit: spatial flows q_L, source flow p_S, sink flows
 * p_L <= D_L, and the labels u_L as the multipliers of flow conservation
 * div q_L - p_S + p_L = 0.  One iteration of the augmented Lagrangian with
 * penalty c = params->c and spatial step tau = params->tau:
 *   q_L <- Proj_{|q_L| <= S_L}(q_L + tau grad(div q_L - p_S + p_L - u_L/c))
 *   p_L  = min(D_L, p_S - div q_L + u_L/c)
 *   p_S <- (1/n) sum_L (div q_L + p_L - u_L/c) + 1/(n c)
 *   u_L <- u_L - c (div q_L - p_S + p_L)
 * from q = 0, p_S = p_L = min_L D_L, u = 1/n_labels.  State (float32 only,
 * in the caller's workspace of pf_fullflow_workspace_bytes): q, u, p_S and
 * the flow-step driver div q_L - p_S + p_L - u_L/c, (ndim + 2) n + 1 fields
 * per voxel.  Energy and dual (float64): E of u clipped at 0 and renormalised
 * per voxel, P = sum_x min_L (D_L + div q_L); max_simplex_err is
 * max |sum_L u_L - 1|.  result->u receives u as it is (it need not be >= 0
 * before convergence), result->labels its argmax, result->q the spatial
 * flows; result->ell must be NULL.  At most 16 labels; storage PF_FP32 and
 * kernel PF_KERNEL_AUTO or PF_KERNEL_TWO_PASS, no tape (PF_EUNSUPPORTED
 * otherwise).  Other arguments, errors, streams and timing as solve_potts. */
size_t pf_fullflow_workspace_bytes(const pf_grid *grid, int32_t n_labels);
int solve_potts_fullflow(const pf_grid *grid, int32_t n_labels, const float *D, const float *S,
                         int32_t s_mode, const pf_params *params, pf_result *result,
                         void *stream);

/* Bytes of checkpoint tape for `iters` iterations recorded every
 * `ckpt_every` iterations (float32 state); 0 for invalid arguments. */
size_t pf_tape_bytes(const pf_grid *grid, int32_t n_leaf, int32_t n_node, int32_t iters,
                     int32_t ckpt_every);

/* Bytes of device workspace for a backward call (segment states, adjoint
 * buffers); 0 for invalid arguments. */
size_t pf_backward_workspace_bytes(const pf_grid *grid, int32_t n_leaf, int32_t n_node,
                                   int32_t ckpt_every);

/* Reverse-mode gradient of a loss on the final log-labels ell_K = ln u_K of
 * a recorded solve (the paper has no gradients; this differentiates its
 * Algorithm 1 / Algorithm 2 iteration as unrolled).  Inputs: the same grid,
 * labels or graph, D, S and s_mode as the recorded call, and `params` with the
 * same iters, c, tau, ckpt_every and tape, `workspace` of at least
 * pf_backward_workspace_bytes.  grad_ell: device float[B][n_leaf][Z][Y][X],
 * dLoss/d ell_K.  Outputs (device, float32, overwritten): grad_D shaped like
 * D; grad_S shaped like S for the field modes, float[n_node] on the device for
 * PF_S_NODE_SCALAR (summed over voxels and problems).  Checkpoint segments
 * are recomputed with the two-pass forward kernels.  params->kernel selects
 * the reverse step: PF_KERNEL_TWO_PASS runs two kernels (projection adjoint,
 * then label adjoint), PF_KERNEL_FUSED one fused kernel (PF_EUNSUPPORTED
 * beyond 8 Potts labels in 2-D, 4 in 3-D, or 4 leaves / 8 flows on a 2-D
 * label graph; not for 3-D label graphs; in 2-D with rows of up to 512
 * voxels it marches along the rows), PF_KERNEL_FUSED2 and PF_KERNEL_LDS
 * PF_EUNSUPPORTED, PF_KERNEL_AUTO the fused kernel where it marches rows and
 * the two kernels otherwise (faster on MI355X).  Both give the same
 * gradients bit for bit.  The tape
 * and the inputs must be those of the recorded call: the library cannot
 * check that.  Calls sharing a workspace must not overlap. */
int pf_potts_backward(const pf_grid *grid, int32_t n_labels, const float *D, const float *S,
                         int32_t s_mode, const pf_params *params, const float *grad_ell,
                         float *grad_D, float *grad_S, void *stream);
int pf_dagmf_backward(const pf_grid *grid, const pf_graph *graph, const float *D,
                         const float *S, int32_t s_mode, const pf_params *params,
                         const float *grad_ell, float *grad_D, float *grad_S, void *stream);

/* Message for the last failing call on this thread ("" if none). */
const char *pf_last_error(void);

/* PF_ABI_VERSION of the loaded library. */
int32_t pf_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PSEUDOFLOW_H */
