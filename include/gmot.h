/*
 * gmot.h -- C ABI of libgmot, a gfx950 (MI355X) solver for tree-structured
 * coupled bi-marginal optimal transport with local entropic regularisation.
 *
 * Method: Fan, Haasler, Zhang, Karlsson, Chen, "A parallel framework for
 * graphical optimal transport" (arXiv 2406.10849), Section 3.  The library
 * runs the Bipartite Iterative Scaling algorithm (Algorithm tree_local_reg) in
 * the log domain: per-edge Gibbs-kernel products K u are computed as
 * log-sum-exp reductions with the cost formed on the fly, every edge that
 * touches one colour class of the tree's 2-colouring is processed
 * concurrently, and the two classes alternate.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Return value: GMOT_OK (0) on success, a negative GMOT_E* code on error.
 *   gmot_strerror() names a code; gmot_last_error() gives a message for the
 *   most recent failure on the calling thread.  Failed calls leave their
 *   outputs unspecified and their handles usable.
 * - Non-convergence is not an error: it is reported in gmot_result.status.
 * - Ownership: the caller owns every input array and may free it as soon as
 *   the call that reads it returns (problem creation deep-copies its inputs
 *   into device memory).  The library owns every handle; *_destroy frees it.
 *   Output arrays are caller-allocated host memory unless a name ends in _dev.
 * - Potentials are log-scalings Lam = log u (the paper's lambda = eps * Lam,
 *   Section 3.2).  Directed-edge order: edge e = (a, b) contributes
 *   Lam_(a,b) (n_a values, over supp(a)) then Lam_(b,a) (n_b values).
 * - Iterations are half-sweeps: one half-sweep updates one colour class (the
 *   paper's counter t).  Every edge carries exactly one message per
 *   half-sweep.
 * - A handle may be used from one thread at a time.
 */
#ifndef GMOT_H
#define GMOT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------- */
#define GMOT_OK         0
#define GMOT_EINVAL    -1   /* not a tree (edge count, cycle, disconnected, self-loop,
                               duplicate edge), n_j < 1, eps <= 0, tol < 0, bad option  */
#define GMOT_EMARGINAL -2   /* a given marginal has a negative entry or |sum - 1| > 1e-9
                               (the library never renormalises silently)               */
#define GMOT_ENOMEM    -3   /* device or host allocation failed                         */
#define GMOT_EDEVICE   -4   /* a HIP call failed, or no gfx950 device is present        */
#define GMOT_ENOTSUP   -5   /* unsupported input (dim outside 1..3, unknown cost kind)   */
#define GMOT_ESTATE    -6   /* handle in the wrong state (e.g. batch of mixed contexts) */

/* ---- solve status (gmot_result.status) ------------------------------------ */
#define GMOT_CONVERGED      0   /* stopping sum <= tol                               */
#define GMOT_NOT_CONVERGED  1   /* max_steps half-sweeps done, sum still > tol       */
#define GMOT_NONFINITE      2   /* a NaN/Inf appeared; the last finite state is kept */

/* ---- cost kinds ------------------------------------------------------------ */
#define GMOT_COST_SQEUCLID  0   /* C(x, y) = |x - y|^2 from the supports, on the fly */
#define GMOT_COST_EXPLICIT  1   /* per-edge cost matrices given as float32           */

/* ---- arithmetic of the message kernel -------------------------------------- */
#define GMOT_PREC_FP32CORE  0   /* FP64 state and exponent arguments, FP32 exp2, FP64
                                   accumulation of FP32 pair sums                     */
#define GMOT_PREC_FP64      1   /* everything in FP64                                  */

typedef struct gmot_ctx gmot_ctx;         /* device, stream, tile-tuning cache        */
typedef struct gmot_problem gmot_problem; /* one tree instance resident in HBM        */
typedef struct gmot_batch gmot_batch;     /* many instances solved in shared launches */

/*
 * One instance of the coupled problem (eq. ot_graph_pairwise_mass):
 *   min sum_e <C_e, B_e> + eps * H(B_e | gamma_a (x) gamma_b)
 * with B_e 1 = mu_a, B_e^T 1 = mu_b, mu_j given on constrained nodes (Gamma)
 * and free (unit mass) elsewhere; gamma_j = mu_j on Gamma, 1 elsewhere
 * (eq. jointdist).  A constrained node of degree r > 1 acts as r constrained
 * leaves with the same marginal (it splits the tree, Section 3.1).
 */
typedef struct {
  int32_t        n_nodes;     /* N >= 1                                                */
  int32_t        n_edges;     /* must be N - 1                                         */
  const int32_t* edges;       /* [2 * n_edges]: (a, b) pairs; B_e is n_a x n_b          */
  const int32_t* sizes;       /* [N]: support size n_j >= 1                             */
  int32_t        dim;         /* D in 1..3 (GMOT_COST_SQEUCLID)                          */
  const double*  support;     /* [sum_j n_j * D], node-major, point-major; may be NULL
                                 for GMOT_COST_EXPLICIT                                  */
  const uint8_t* is_fixed;    /* [N]: 1 if j in Gamma                                   */
  const double*  marginal;    /* given marginals of constrained nodes, concatenated in
                                 node order ([sum_{j in Gamma} n_j]); entries >= 0 and
                                 each block sums to 1 within 1e-9                        */
  int32_t        cost_kind;   /* GMOT_COST_*                                             */
  const float*   cost;        /* GMOT_COST_EXPLICIT: per-edge n_a x n_b row-major
                                 matrices concatenated in edge order                    */
  double         eps;         /* regularisation, > 0                                    */
} gmot_tree_desc;

typedef struct {
  double  tol;          /* stop at the first half-sweep t >= 2 whose stopping sum
                           (Algorithm tree_local_reg) is <= tol; >= 0                  */
  int64_t max_steps;    /* at most this many half-sweep updates (> 0)                  */
  int32_t check_every;  /* half-sweeps per launched graph (even, >= 2; 0 = default)   */
  int32_t precision;    /* GMOT_PREC_*                                                  */
  int32_t restart;      /* 1: start from u = 1 (cold); 0: continue from the held state
                           (after gmot_set_potentials, or a previous solve)            */
  int32_t timing;       /* 1: launch the half-sweeps directly on the stream (not as a
                           captured graph) with HIP events around every message and
                           node stage, and accumulate the stage durations (read with
                           gmot_*_stats); 0: graph replay, no events                  */
  int32_t skip_verify;  /* GMOT_PREC_FP32CORE only.  0 (default): the FP32-core loop
                           runs until its own stopping sum is <= 0.8 * tol, or until
                           that sum has not come 3% below its last record for 64
                           half-sweeps (FP32 noise floor above tol), then FP64
                           half-sweeps continue
                           within the remaining max_steps until the FP64 stopping sum
                           is <= tol, so convergence is judged in FP64.  1: stop on
                           the FP32-core sum <= tol.                                 */
  int32_t schedule;     /* GMOT_SCHED_LAYER (default): every message of the class being
                           updated in one launch; GMOT_SCHED_PER_NODE: the same
                           half-sweep with one launch per node, issued node after
                           node (same iterates); GMOT_SCHED_GAUSS_SEIDEL (gmot_solve
                           only): node-sequential sweeps -- every node, in
                           breadth-first order from node 0, takes the per-node
                           update of Algorithm tree_local_reg from its neighbours'
                           latest potentials -- always in FP64; the stop test is the
                           stopping sum over every node, before the first sweep and
                           after every check_every sweeps (0: 4); result.steps counts
                           sweeps, max_steps bounds them, t is left unchanged; a
                           non-finite sum stops with GMOT_NONFINITE without rollback */
  int32_t msg_passes;   /* FP32-core message sums.  GMOT_PASSES_AUTO (0, default): two
                           passes (row max, then sum) for the first two half-sweeps of
                           the call, then one pass shifted by each row's max from the
                           previous computation of the same message, with in-kernel
                           re-shifting when a row leaves the FP32 range; the sums are
                           exact either way.  GMOT_PASSES_ONE (1): one pass from the
                           first half-sweep, shifted by the maxima of the plan's last
                           computation (0 before any).  GMOT_PASSES_TWO (2): always two
                           passes. */
} gmot_opts;

#define GMOT_PASSES_AUTO  0
#define GMOT_PASSES_ONE   1
#define GMOT_PASSES_TWO   2

#define GMOT_SCHED_LAYER         0
#define GMOT_SCHED_PER_NODE      1
#define GMOT_SCHED_GAUSS_SEIDEL  2

/* Kernel timing accumulated by solves with opts.timing = 1 (since the last
 * reset).  Only half-sweeps that did work for at least one instance count. */
typedef struct {
  double  msg_ms;          /* summed duration of the node-kernel stages (messages, terms
                              and update; ms), each the mean of 4 back-to-back repeats of
                              the stage (each repeat rewrites the same slots from the
                              same state), so event overhead is not counted             */
  double  sweep_ms;        /* summed duration of whole half-sweeps: node stage and
                              finalise kernel (ms)                                     */
  int64_t msg_launches;    /* half-sweeps timed                                         */
  double  msg_pairs;       /* (x, y) terms those half-sweeps evaluated: n_j n_k per
                              message, A_k B_j B_k + n_j A_k per separable one (grid
                              supports of A rows and B columns)                         */
  int64_t graph_launches;  /* graph replays issued (timed or not)                        */
  double  group_ms[7];     /* the node stage split by kernel group (explicit cost;
                              D = 1, 2, 3; separable grids; uniform 1D grids; separable
                              uniform grids), each the mean of 4 back-to-back repeats
                              of the group alone, summed (ms)                           */
  double  group_pairs[7];  /* the terms each group evaluated in those half-sweeps        */
} gmot_stats;

typedef struct {
  int32_t status;        /* GMOT_CONVERGED / GMOT_NOT_CONVERGED / GMOT_NONFINITE         */
  int32_t reserved;
  int64_t steps;         /* half-sweep updates applied by this call                      */
  int64_t t;             /* the paper's counter after the call (state = before step t)  */
  double  err_sum;       /* stopping sum of the returned state (as measured in-loop)     */
  double  err_max;       /* largest single per-edge term of that sum                     */
  double  seconds;       /* device time from the first half-sweep to the stop decision   */
} gmot_result;

/* Objective values of the current state, computed in FP64 on the device
 * (definitions: dual = -eps * f(u, rho) of eq. tree_dual_mass_consv; primal =
 * sum_e <C_e,B_e> + eps H(B_e|M_e) with the -1 term of eq. entropy_term;
 * transport = sum_e <C_e, B_e>; the stopping sum over both colour classes). */
typedef struct {
  double dual, primal, transport, gap;   /* gap = primal - dual                        */
  double err_sum, err_max;               /* stopping sum over every node, largest term */
  double mass_min, mass_max;             /* extremes of ||B_e||_1 over edges            */
  double rho_spread;                     /* max over free nodes of the spread in x of
                                            sum_k Lam_(j,k)(x) (0 at exact iterates)   */
  double scale;                          /* sum |eps <Lam, mu>| + sum |eps rho| + eps|E|,
                                            the scale for relative dual comparisons    */
} gmot_eval;

/* ---- context ---------------------------------------------------------------- */
/* Bind device `device`; `hip_stream` (a hipStream_t, may be NULL) is the stream
 * every launch is ordered on; NULL makes the library create its own. */
int  gmot_ctx_create(gmot_ctx** out, int device, void* hip_stream);
/* Drop the caller's reference.  Every live problem, batch and network holds
 * one more, so the context (stream, scratch) is freed when the last of them is
 * destroyed: handles may be destroyed in any order. */
void gmot_ctx_destroy(gmot_ctx* ctx);

/* ---- problems ----------------------------------------------------------------- */
/* Validate `desc` (GMOT_EINVAL / GMOT_EMARGINAL / GMOT_ENOTSUP) and copy it to the
 * device.  The tree is 2-coloured by BFS from node 0; `first_color` (0 or 1, or -1
 * for the class of node 0) selects which class the first half-sweep updates.
 * The potentials start at Lam = 0 (u = 1). */
int  gmot_problem_create(gmot_ctx* ctx, const gmot_tree_desc* desc, int32_t first_color,
                         gmot_problem** out);
void gmot_problem_destroy(gmot_problem* p);

/* Run Algorithm tree_local_reg until the stopping sum of the current state is
 * <= opts->tol (check-then-update: the returned state is the one that passed)
 * or opts->max_steps updates were applied. */
int  gmot_solve(gmot_problem* p, const gmot_opts* opts, gmot_result* out);

/* FP64 objective values and the both-side stopping sum of the held state. */
int  gmot_evaluate(gmot_problem* p, gmot_eval* out);

/* Number of doubles in the potential vector (sum_e n_a + n_b). */
int64_t gmot_potentials_size(const gmot_problem* p);
/* Copy the held potentials out / in (directed-edge order above).  Setting them
 * makes the next gmot_solve with restart = 0 continue from them (warm start,
 * or resume from a checkpoint); the counter t restarts at 1. */
int  gmot_get_potentials(gmot_problem* p, double* out);
int  gmot_set_potentials(gmot_problem* p, const double* in);
/* Device-pointer variants, ordered on the context stream, no implicit sync. */
int  gmot_get_potentials_dev(gmot_problem* p, double* out_dev);
int  gmot_set_potentials_dev(gmot_problem* p, const double* in_dev);

/* Plan B_e (eq. bi-marginal_B_sol) of edge `edge`, n_a x n_b row-major, FP64. */
int  gmot_get_coupling(gmot_problem* p, int32_t edge, double* out);
/* q_bar_j: arithmetic mean over neighbours k of B_(j,k) 1 (n_j values). */
int  gmot_get_node_marginal(gmot_problem* p, int32_t node, double* out);

/* ---- general graphs: modified junction trees -------------------------------------
 * Coupled MOT on a modified junction tree (Section 4: Definition jt_general,
 * eq. ot_graph_local_reg): separators alternate with cost cliques, every cost
 * clique has exactly two neighbouring separators, and the separator--clique
 * graph is a tree (n_cliques = n_seps - 1, connected).  Supported class: each
 * clique's variables are the variables of its two separators (every variable
 * belongs to exactly one separator, so the two sets are disjoint), and a
 * constraint fixes the joint marginal of all of a separator's variables.  The
 * Wasserstein least-squares problem of Section 2 on its modified junction tree
 * is of this class.  Every intersection of a separator with a neighbouring
 * clique is then the separator itself, and the separator update of
 * Proposition general_algo becomes the node update of Algorithm
 * tree_local_reg on the tree whose nodes are the separators: node s has one
 * state per joint state of its variables (C order over them), edge c carries
 * the clique's cost tensor read as a (states of a) x (states of b) matrix.
 * The library builds that problem (explicit FP32 costs) and returns it as an
 * ordinary gmot_problem: gmot_solve, gmot_evaluate, the batch calls and the
 * potential, coupling and node-marginal read-backs apply, in clique order for
 * potentials (log u of separator a, then of b, per clique), with couplings =
 * clique plans B_c as (states of a) x (states of b) matrices and node
 * marginals = separator marginals.  The caller owns every array. */
typedef struct {
  int32_t        n_vars;       /* variables, >= 1                                             */
  const int32_t* var_sizes;    /* [n_vars]: support size of each variable, >= 1                */
  int32_t        n_seps;       /* separators, >= 1                                            */
  const int32_t* sep_nvars;    /* [n_seps]: variables of each separator, >= 1                  */
  const int32_t* sep_vars;     /* concatenated variable indices of the separators, in tensor-axis
                                  order; every variable appears exactly once                  */
  const uint8_t* sep_fixed;    /* [n_seps]: 1 if the separator's joint marginal is given        */
  const double*  sep_marginal; /* joint marginals of the fixed separators, concatenated in
                                  separator order, each in C order over its variables; entries
                                  >= 0, each sums to 1 within 1e-9                             */
  int32_t        n_cliques;    /* cost cliques, = n_seps - 1                                  */
  const int32_t* cliques;      /* [2 * n_cliques]: the two neighbouring separators (a, b)      */
  const float*   clique_cost;  /* concatenated cost tensors C_c over (variables of a, variables
                                  of b), C order, in clique order                              */
  double         eps;          /* regularisation, > 0                                         */
} gmot_junction_desc;

/* Validate `desc` (GMOT_EINVAL: a variable in no or several separators, a bad
 * size, a clique count or pair that does not form a tree, more than 2^31 - 1
 * joint states in a separator; GMOT_EMARGINAL as for trees) and create the
 * problem.  first_color as in gmot_problem_create (separator 0's class by
 * default). */
int  gmot_junction_create(gmot_ctx* ctx, const gmot_junction_desc* desc, int32_t first_color, gmot_problem** out);

/* ---- rounding (Algorithm round) -------------------------------------------------- */
/* After a half-sweep the class S that was not updated last (the one the next
 * half-sweep would update) misses its marginals.  gmot_round rounds every plan
 * B_(j,k), j its end in S, with the rounding of Altschuler, Weed and Rigollet
 * (NeurIPS 2017, Algorithm 2) onto the plans with row marginal r_j (mu_j for a
 * constrained node, the arithmetic mean q_bar_j of the node's plan marginals
 * for a free node) and column marginal B_(j,k)^T 1, so that every node's
 * marginals agree on all its edges and equal mu_j where constrained.  The
 * state is not changed; all arithmetic is FP64 on the device.  Lemma round
 * bounds |transport - unrounded transport| by 2 c_inf err_side.
 * Requires a state produced by at least one half-sweep (t >= 2; otherwise
 * GMOT_ESTATE): unit plan mass (Lemma tree_mass) is what makes the rounded
 * marginals exact. */
typedef struct {
  double  transport;   /* sum_e <C_e, G_e> over the rounded plans G_e                    */
  double  err_side;    /* sum over j in S, k in N(j) of |r_j - B_(j,k) 1|_1              */
  double  c_inf;       /* max |C| over all pairs of all edges                            */
  int32_t side;        /* S: 0 = the class updated on odd half-sweeps, 1 = the other      */
  int32_t reserved;
} gmot_round_result;

/* edge_transport: optional host array of n_edges, <C_e, G_e> per edge.
 * Keeps device buffers (4 doubles per potential entry) until the state changes. */
int  gmot_round(gmot_problem* p, gmot_round_result* out, double* edge_transport);
/* G_e of the last gmot_round of the held state, n_a x n_b row-major, FP64 (host
 * array).  GMOT_ESTATE if the state changed since (or no rounding was done). */
int  gmot_get_rounded_coupling(gmot_problem* p, int32_t edge, double* out);

/* ---- batches ------------------------------------------------------------------ */
/* Group `count` problems of one context so that every half-sweep of all of them
 * runs in the same launches; instances converge independently (a converged
 * instance stops updating and keeps its passing state).  The batch works on
 * its problems' device buffers: keep them alive while the batch is used (its
 * destroy call touches none of them, so it may come before or after theirs). */
int  gmot_batch_create(gmot_ctx* ctx, gmot_problem* const* probs, int32_t count, gmot_batch** out);
void gmot_batch_destroy(gmot_batch* b);
/* outs: [count] results, one per instance. */
int  gmot_batch_solve(gmot_batch* b, const gmot_opts* opts, gmot_result* outs);
/* gmot_evaluate for every instance of the batch, in shared launches: the FP64
 * messages into both classes, the node terms and the pair pass of all
 * instances run as one set of launches, each instance read from its own held
 * state.  outs: [count]; the values equal per-instance gmot_evaluate calls up
 * to the order in which column splits of a message are added (the split count
 * depends on how many messages share the launch). */
int  gmot_batch_evaluate(gmot_batch* b, gmot_eval* outs);

/* ---- learned warm start ------------------------------------------------------------
 * Not part of the paper's method: a small network predicts starting potentials
 * for star instances; the bipartite iteration then runs as usual and still
 * decides convergence (a cold start is the fallback).  For the callers
 * that want fewer half-sweeps on families of similar barycenter problems. */
typedef struct gmot_mlp gmot_mlp;

/* Fully connected network widths[0] -> ... -> widths[n_layers], ReLU between
 * layers, linear output.  GEMM inputs are rounded to BF16 (nearest even) and
 * accumulated in FP32 on the matrix cores; parameters, activations, Adam
 * moments and the loss are FP32.  Every width must be a multiple of 8
 * (GMOT_ENOTSUP otherwise).  Weights are He-uniform from `seed`, biases 0. */
int  gmot_mlp_create(gmot_ctx* ctx, int32_t n_layers, const int32_t* widths, uint64_t seed, gmot_mlp** out);
void gmot_mlp_destroy(gmot_mlp* m);
int64_t gmot_mlp_num_params(const gmot_mlp* m);
/* FP32 parameters, layer by layer: W_l (widths[l] x widths[l-1], row-major), b_l.
 * Setting them also clears the Adam state. */
int  gmot_mlp_get_params(gmot_mlp* m, float* out);
int  gmot_mlp_set_params(gmot_mlp* m, const float* in);
/* Device buffers, row-major FP32: x [batch x widths[0]], y [batch x widths[n]];
 * batch must be a positive multiple of 8.  Stream-ordered on the context. */
int  gmot_mlp_forward_dev(gmot_mlp* m, const float* x_dev, int32_t batch, float* y_dev);
/* The same forward pass with no allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The activations live in a static device workspace
 * of 16 MiB per device (held until the process ends) instead of the network's
 * own buffers: 2 * batch * widths[0] bytes for the BF16 input, then
 * 6 * batch * widths[l] bytes per hidden layer, then the split-K partial sums
 * of the widest layer product (4 * s * batch * widths[l] bytes when a layer's
 * K is split in s parts: s doubles while the 64 x 64 output tiles times 2s
 * stay within 512 blocks and each part keeps at least 512 of K), each part
 * aligned to 256 bytes; a batch that does not fit returns GMOT_EINVAL (the message
 * gives the batches that fit).  Nothing in it needs clearing: every part is
 * written before it is read.  Results equal gmot_mlp_forward_dev's.  All calls
 * on one device share the workspace: calls ordered on one stream are safe,
 * calls that overlap on one device (other streams, other contexts, other
 * threads) race.  Stream-ordered on the context stream, no synchronisation. */
int  gmot_mlp_forward_static(gmot_mlp* m, const float* x_dev, int32_t batch, float* y_dev);
/* Mean-squared-error loss sum (y - t)^2 / (batch * widths[n]) (host, after a
 * sync; may be NULL) and its FP32 parameter gradient (device, parameter layout;
 * may be NULL) for targets t_dev [batch x widths[n]]. */
int  gmot_mlp_loss_grad_dev(gmot_mlp* m, const float* x_dev, const float* t_dev, int32_t batch, double* loss,
                            float* grad_dev);
/* Bias-corrected Adam step with the gradient of the last loss_grad call. */
int  gmot_mlp_adam_step(gmot_mlp* m, float lr, float beta1, float beta2, float adam_eps);
/* loss_grad followed by Adam(lr, 0.9, 0.999, 1e-8). */
int  gmot_mlp_train_step_dev(gmot_mlp* m, const float* x_dev, const float* t_dev, int32_t batch, float lr,
                             double* loss);
const char* gmot_mlp_last_error(void);

/* Star instances for the warm start: node 0 is a free center, edges are
 * (0,1), (0,2), ..., (0,L) in that order, leaves 1..L are constrained, every
 * support has the same size n, and all instances of one call share L and n.
 *   features: x[i][l*n + p] = (max(log mu_l(p), -40) - shift) * scale
 *   targets:  t[i][l*n + p] = (Lam_(l,0)(p) - mean_p Lam_(l,0)) / out_scale, from
 *             the held (committed) potentials
 *   apply:    Lam_(l,0) = out_scale * (y_l - mean_p y_l), Lam_(0,l) = 0 become the
 *             held potentials (t restarts at 1, the center is updated first);
 *             an instance whose prediction has a non-finite entry gets the cold
 *             start instead and is counted in *rejected. */
int  gmot_star_features_dev(gmot_problem* const* probs, int32_t count, float shift, float scale, float* x_dev);
int  gmot_star_targets_dev(gmot_problem* const* probs, int32_t count, float out_scale, float* t_dev);
int  gmot_star_apply_dev(gmot_problem* const* probs, int32_t count, const float* y_dev, float out_scale,
                         int32_t* rejected);
/* features -> forward -> apply in one call, with library-owned workspaces. */
int  gmot_mlp_warm_start(gmot_mlp* m, gmot_problem* const* probs, int32_t count, float shift, float scale,
                         float out_scale, int32_t* rejected);

/* ---- tile autotuning ------------------------------------------------------------ */
/* Time the candidate node-kernel block shapes (2, 4, 8 or 16 waves per tile, the
 * waves splitting each edge's source columns; 1 or 2 rows per lane; 1 or 2 lane
 * groups per wave, the groups of a wave splitting its columns again; tiles of
 * 64 * rows_per_lane / lane_groups = 32, 64 or 128 rows) by the device time of a
 * few real FP32-core half-sweeps (node stage and finalise kernel) run from a
 * snapshot of the held state, which is restored afterwards, and keep the
 * fastest plan; best_ms is that half-sweep time.
 * The choice is cached in the context under the instances' shapes, so later
 * problems or batches of the same shapes start with it.  Outputs may be NULL. */
int  gmot_problem_autotune(gmot_problem* p, int32_t* waves_per_block, int32_t* rows_per_lane,
                           int32_t* lane_groups, double* best_ms);
int  gmot_batch_autotune(gmot_batch* b, int32_t* waves_per_block, int32_t* rows_per_lane,
                         int32_t* lane_groups, double* best_ms);

/* ---- diagnostics ----------------------------------------------------------- */
/* Copy out (and, if reset != 0, clear) the kernel timing of a problem's own
 * solves or of a batch's solves. */
int  gmot_problem_stats(gmot_problem* p, gmot_stats* out, int32_t reset);
int  gmot_batch_stats(gmot_batch* b, gmot_stats* out, int32_t reset);
const char* gmot_strerror(int code);
const char* gmot_last_error(void);
/* Node-kernel shape of the most recent plan: rows per block (64 or 128), waves per
 * block, and blocks per half-sweep for each class. */
int  gmot_last_tiles(int32_t* rows_per_block, int32_t* waves_per_block, int32_t* blocks_c0, int32_t* blocks_c1);

#ifdef __cplusplus
}
#endif
#endif /* GMOT_H */
