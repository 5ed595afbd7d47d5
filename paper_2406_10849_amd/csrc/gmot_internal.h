// Device-side tables shared by the HIP kernels and the host runtime of libgmot.
//
// Notation (Section 3 of the paper): every edge e = (a, b) carries two
// log-scalings, Lam_(a,b) over supp(a) and Lam_(b,a) over supp(b) ("directed
// edges").  At half-sweep t the class S being updated receives one message
// per incident edge,
//     m_{k->j}(x) = log sum_y K_(j,k)(x, y) u_(k,j)(y) gamma_k(y)
//                 = LSE_y [ Lam_(k,j)(y) + log gamma_k(y) - C(x, y) / eps ],
// which is log of the product K (u * gamma) in Theorem tree_dual_var.  The
// message kernel evaluates it in base 2 as
//     w(x, y) = a(y) + sum_d c_d(x) y_d,   a(y) = log2e (Lam + log gamma - |y|^2/eps),
//     c_d(x) = 2 log2e x_d / eps,          m(x) = ln2 * log2 sum_y 2^w - |x|^2 / eps
// for the squared-Euclidean cost, and w = log2e (Lam + log gamma - C / eps)
// for explicit cost matrices.
//
// Potentials are double-buffered by update count: the k-th update of a node
// writes slot k % 2.  Before half-sweep t the class updated at t holds its
// value in slot ((t - 1) / 2) % 2 and the other class in slot (t / 2) % 2, so a
// half-sweep that ends in "converged" has written only the slot nobody reads
// and the state that passed the test stays intact (check-then-update).
//
// A free node's potentials are held as Lam_(j,k)(x) = L_(j,k)(x) - c_j: the
// update writes L = abar - m_{k->j} row tile by row tile, and the node-wide
// normaliser c_j = LSE_x abar is written once all tiles are done (constrained
// nodes have c_j = 0).  c_j is double-buffered like the potentials.
//
// One half-sweep is two stream-ordered launches: the node kernel (one block
// per 64-row tile of every node of the class, per support dimension: the
// messages of all incident edges for those rows, the stopping-sum terms of the
// state before the update, the update of L, and a tile record) and the
// finalise kernel (one block per instance: c_j from the tile records, the
// stopping sum and the stop decision).  The kernel boundary makes the tiles'
// writes visible to the finalise kernel, so no block waits on, or fences for,
// another block.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace gmot {

constexpr int kBlock = 256;          // threads per block, every kernel
constexpr int kChunk = 256;          // columns staged in LDS per chunk (one per thread)
constexpr double kLog2e = 1.44269504088896340736;
constexpr double kLn2 = 0.693147180559945309417;

enum Done : int { kRunning = 0, kConverged = 1, kMaxSteps = 2, kNonFinite = 3, kStalled = 4 };

// Potential slots per class: a class's held potentials after its u-th update
// are in slot u mod kSlots, so the two states before any update stay intact.
constexpr int kSlots = 3;

// One message m_{k->j}: rows index supp(j) ("dst"), columns index supp(k) ("src").
struct MsgDesc {
  const double* supp_dst;    // [n_dst * dim]
  const double* supp_src;    // [n_src * dim]
  const double* lam_src[kSlots];  // stored L_(k,j) slots, [n_src]
  const double* c_src;       // c_k slots [kSlots] (NULL: constrained source, c = 0)
  const double* lg_src;      // log gamma_k, [n_src]
  double* lam_dst[kSlots];   // stored L_(j,k) slots, [n_dst]
  double2* partial;          // [n_dst * ns]: evaluation pass, per row its ns column splits, each
                             // (split max M, sum of 2^(w - M))
  double* wmax;              // [kMaxRanges * n_dst]: node kernel, wave-major, per row the max (to
                             // within one binade) of each wave's column range at the last
                             // computation (next shift)
  double* mfull;             // merged message m_{k->j}, [n_dst], natural log
  const float* cost;         // explicit cost stored src-major: cost[y * n_dst + x] = C_(j,k)(x, y)
  const float* cost_tile;    // the same, tile-major for the node kernel: C_(j,k)(x, y) at
                             // ((x / 64) * n_src + y) * 64 + x % 64, rows padded to 64
  const double* src_tpart;   // tile records of the source node k (its c_k comes from them)
  double* sepT;              // separable messages (grid supports): first-pass sums, transposed,
                             // Tt(q, u) = T(u, q) - kap R_k[u]^2 at q * rows_src + u (log2), else NULL
  double* sepM;              // separable messages, [rows_src x cols_dst]: first-pass shifts (log2 max
                             // term) of k_sep_pass; in k_sep_horner's evaluation mode, at Tt's index,
                             // the first pass's mean of (C_j[q] - C_k[i])^2 under the line's weights
  int32_t n_dst, n_src, ns, inst;
  int32_t dim, cost_kind, src_tiles, src_deg;  // source node's tile count and degree
  int32_t src_free;          // 1: free source node (c_k from the records), 0: c_k = 0
  int32_t grid;              // 1: the message is summed by k_msg_grid or k_sep_horner (whose evaluation
                             // modes leave in wmax[x] the mean cost of row x under the plan's row:
                             // sum_y B C / sum_y B)
  int32_t pad1, pad2;
  int32_t rows_src, cols_src, rows_dst, cols_dst;  // grid shapes of both supports (separable messages)
  double eps;
};

// One block of a separable pass: lines [line0, line0 + nlines) of message msg
// (source grid rows in the first pass, destination grid columns in the second).
struct SepItem {
  int32_t msg, line0, inst, nlines;
};
// One wave of a separable pass on uniform grids (k_sep_horner): outputs
// [o0, o0 + 64) of lines [line, line + kSepLines) of message msg.
struct SepTask {
  int32_t msg, line, o0, inst;
};
constexpr int kSepTaskLines = 8;  // lines per SepTask (the kernel's kSepLines)
constexpr int kSepWaves = 4;        // waves per block of a separable pass
constexpr int kSepMaxSide = 2048;   // grid rows and columns of a separable support at most
constexpr int kSepMaxOut = 2048;    // outputs per separable-pass block (8 per thread)
constexpr int kSepStage = 4608;     // staged values per separable-pass block (36 KB) at most
// Messages from uniform one-dimensional grids sum a polynomial in each row's
// ratio rho; the host admits a message only when every power of rho it takes
// lies within 2^(+-kGridRange).  With the column values v_j <= 2^kGridSlack
// (128) the sums stay below 2^(11 + 128 + 850) = 2^989, and a v_j lost below
// the FP64 range (2^-1074) is a term below 2^(-1074 + kGridRange) = 2^-224 of
// the row's largest one (at least 2^-G when rho < 1, at least 1 otherwise).
constexpr double kGridRange = 850.0;
constexpr double kGridSlack = 128.0;  // the kernels keep v_j = 2^(C(j) - theta) <= 2^kGridSlack
// Staged row stride and length of a separable pass with `inner` terms per output.
__host__ __device__ inline int sep_row_stride(int inner) { return (inner + 1) | 1; }
__host__ __device__ inline int sep_inner_even(int inner) { return (inner + 1) & ~1; }

// One block of the message kernel: rows [row0, row0 + rows per block) of a
// message, columns [col0, col0 + ncols), writing column split `split`.
struct K1Item {
  int32_t msg, row0, col0, ncols, split, inst, pad0, pad1;
};

constexpr int kNodeRowsLane = 64;  // rows per node-kernel tile per row-per-lane (tile = 64 * R rows)
constexpr int kMaxWaves = 16;   // waves per node-kernel block: 2, 4, 8 or 16
constexpr int kMaxRanges = 2 * kMaxWaves;  // column ranges per edge in one node-kernel block
constexpr int kRecExtra = 2;    // tile record entries after the per-edge terms

// One node of the class being updated; its deg incoming messages are
// msgs[msg0 .. msg0 + deg) in ascending neighbour order.  Its rows form
// `tiles` tiles of 64 R rows; tile records (deg stopping-sum terms, then the
// tile's LSE max and scaled sum of abar) start at tpart + tile * (deg + kRecExtra).
struct NodeItem {
  int32_t inst, node, n, deg;
  int32_t fixed, msg0, err_idx, tiles;  // tiles: tile records, one per min(tile rows, 64) rows
  const double* lg;          // log gamma_j, [n]
  const double* mu;          // mu_j for constrained nodes, else NULL
  double* abar;              // scratch [n]: mean_k m_{k->j}
  double* qbar;              // scratch [n]: arithmetic mean_k q_(j,k)
  double* c;                 // c_j slots [kSlots] (NULL for constrained nodes)
  double* tpart;             // tile records
};

// One block of the node kernel: rows [row0, row0 + 64 R / H) of node item
// `node` of instance `inst`.  The node's first message, degree, size and
// kind are repeated here so the instance state, the node item and the message
// descriptors all load one step after the tile item.  msg_only = 1: messages
// msg0 .. msg0 + deg of the node (a subset of its edges) are summed and
// written to mfull, and the node's update is left to k_node_sep.
struct TileItem {
  int32_t node, row0, inst, msg0;
  int32_t deg, n, fixed, msg_only;
};

// Per-instance loop state, written only by the last node block of a half-sweep.
struct InstState {
  long long t;               // next half-sweep; the held state is "before step t"
  long long updates;         // updates applied since the solve started
  long long max_updates;
  double tol;
  double err_sum, err_max;   // stopping sum of the last checked state
  long long checked_t;       // the half-sweep whose state the sum above measures
  long long min_check_t;     // the stop test applies from this half-sweep on
  int done;                  // Done
  int counter;               // node blocks finished in the current half-sweep
  int node0[2], nnodes[2];   // node-error index ranges per class
  unsigned long long clk_start, clk_stop;
  long long onepass_from;    // the FP32-core message kernel runs one pass from this half-sweep on
  double best_err;           // last stopping sum of this call that set a record (3% below the previous one)
  long long best_t;          // the half-sweep that measured it
  long long stall_window;    // stop as stalled after this many half-sweeps without a record (0: never)
  long long t_first;         // first half-sweep of this run: tile records are this run's from t_first on
  // What the node blocks of a colour-c launch read (the fields above are
  // written by the finalise step, which can run in the same launch): the
  // half-sweep they compute, and whether the instance has stopped.
  long long vt[2];
  int vdone[2];
};

struct Tables {
  const MsgDesc* msgs;
  const K1Item* items;       // items of one class and one dimension (kernel argument slice)
  const NodeItem* nodes;     // node items of one class
  const TileItem* tiles;     // tile items of one class
  InstState* inst;
  double4* node_eval;        // evaluation pass: (err sum, err max, <Lam,mu> or rho, spread)
  int* ndone;                // number of instances that reached a final state
  int colour;                // class whose items / nodes these are
  // finalise step carried by a node-kernel launch: its first n_fin blocks
  // decide, per instance, the half-sweep of class fin_colour whose records the
  // previous launch wrote (fin_nodes: that class's node items); 0: none
  int n_fin, fin_colour;
  const NodeItem* fin_nodes;
  const SepItem* sep_items;  // separable first pass of one class
  const SepItem* sep_items2; // separable second pass of one class
  const SepTask* sep_tasks;  // separable first pass on uniform grids (k_sep_horner)
  const SepTask* sep_tasks2; // separable second pass on uniform grids
  int rec_rows;              // rows per tile record (32 or 64)
  // evaluation pass: per instance the slot holding each class's committed
  // potentials, [2 * inst + class] (read when a kernel is given slot -1)
  const int* inst_slot;
  // evaluation pass, per plan message into node j: (sum_x q, sum_x q (L - c_j),
  // sum_x q Cbar, 0) with q the plan's marginal on j and Cbar its row's mean
  // cost (grid messages only, else 0)
  double4* msg_eval;
};

// Pair pass of the evaluation (transport, entropy, mass of each plan).
struct EdgeDesc {
  const double* supp_a;  const double* supp_b;
  const double* lam_a;   const double* lam_b;     // committed slots of L_(a,b), L_(b,a)
  const double* c_a;     const double* c_b;       // committed c of a and b (NULL: 0)
  const double* lg_a;    const double* lg_b;
  const float* cost;                              // explicit, row-major n_a x n_b, or NULL
  int32_t n_a, n_b, dim, cost_kind;
  double eps;
};
struct PairItem { int32_t edge, row0, col0, ncols; };

// Rounding (Algorithm round): one directed edge (j, k) seen with rows on j.
struct RoundDesc {
  const double* supp_r;  const double* supp_c;    // supports of j (rows) and k (columns)
  const double* lam_r;   const double* lam_c;     // committed L_(j,k), L_(k,j)
  const double* c_r;     const double* c_c;       // committed c_j, c_k (NULL: 0)
  const double* lg_r;    const double* lg_c;
  const float* cost;                              // explicit: cost[y * n_r + x] = C(x, y); else NULL
  double* rs;            // [n_r] row sums B1 (pass 0)
  double* tg;            // [n_r] row target r (rows in S)
  double* sc;            // [n_r] row scaling: X (rows in S) or Y (rows on the other side)
  double* er;            // [n_r] residual: e_r (rows in S) or e_c
  const double* sc_col;  // [n_c] column scaling of the pass (NULL: 1)
  const double* er_col;  // [n_c] e_c of the columns (pass 2)
  int32_t n_r, n_c, dim, cost_kind;
  double eps;
};
struct RoundItem { int32_t desc, row0; };
// A node of S; its directed edges are descs d0 .. d0 + deg.
struct RoundNode {
  int32_t n, deg, d0, pad;
  const double* mu;      // mu_j for constrained nodes, else NULL
};

// ---- launch wrappers (defined in gmot_kernels.hip) ----
// FP64 evaluation messages from potential slot src_slot of the source class
// (-1: each instance's committed slot, from tb.inst_slot)
hipError_t launch_msg(const Tables& tb, int n_items, int dim, int rows_per_lane, int src_slot, hipStream_t s);
// node kernel over n_tiles tiles of one class and support-dimension group (dim 0: explicit
// cost); tiles of 64 * rows_per_lane / lane_groups rows, each wave's lanes in lane_groups
// groups that sum separate column ranges (1, or 2 with two rows per lane)
hipError_t launch_node(const Tables& tb, int n_tiles, int dim, int waves, int rows_per_lane, int lane_groups,
                       bool fp64, hipStream_t s);
hipError_t launch_finalize(const Tables& tb, int n_inst, hipStream_t s);
// separable messages on Cartesian grid supports (D = 2): pass 0 over the
// n_items blocks of tb.sep_items (carrying tb.n_fin finalise blocks), pass 1
// over those of tb.sep_items2 (lds_bytes of dynamic LDS per block: the largest
// item's staged values and coordinates), then the node stage over n_tiles
// 64-row tiles
hipError_t launch_sep_pass(const Tables& tb, int pass, int n_items, size_t lds_bytes, bool fp64, hipStream_t s);
hipError_t launch_node_sep(const Tables& tb, int n_tiles, hipStream_t s);
// separable pass `pass` on uniform grids over the n_tasks tasks of
// tb.sep_tasks (pass 0, carrying tb.n_fin finalise blocks) or tb.sep_tasks2
// (pass 1), one wave each; eval as for launch_msg_grid
hipError_t launch_sep_horner(const Tables& tb, int pass, int n_tasks, bool eval, hipStream_t s);
// messages on uniform one-dimensional source grids: one wave per tile item of
// tb.tiles (a message, msg0, for 64 * rows_per_lane destination rows from
// row0; rows_per_lane 1 or 2), writing mfull; the first tb.n_fin blocks carry
// the finalise step.  eval: the FP64 evaluation pass (committed slots from
// tb.inst_slot, every item, the message as column split 0 of md.partial)
hipError_t launch_msg_grid(const Tables& tb, int n_items, int rows_per_lane, bool eval, hipStream_t s);
hipError_t launch_node_eval(const Tables& tb, int n_nodes, int slot, hipStream_t s);
// node-sequential update of node item `node_item` of tb's class from the
// message partials k_msg wrote, into potential slot `slot` (one block)
hipError_t launch_gs_update(const Tables& tb, int node_item, int slot, hipStream_t s);
// dst[i] = src[i] - (c ? *c : 0) over segments (potential read-back on the device)
struct SegCopy { const double* src; double* dst; const double* c; int64_t len; };
hipError_t launch_seg_copy(const SegCopy* segs, int n_segs, hipStream_t s);
hipError_t launch_stamp(InstState* inst, int count, hipStream_t s);
// dst[0 .. len) = 0 for every segment (a batch's cold restart in one launch)
struct ZeroSeg { double* dst; int64_t len; };
hipError_t launch_zero_segs(const ZeroSeg* segs, int n_segs, hipStream_t s);
hipError_t launch_pairs(const EdgeDesc* edges, const PairItem* items, int n_items, double4* out, hipStream_t s);
hipError_t launch_coupling(const EdgeDesc* edge, double* out, size_t total, hipStream_t s);

// ---- rounding (defined in gmot_round.hip) ----
hipError_t launch_round_rows(int pass, const RoundDesc* ds, const RoundItem* items, int n_items, double4* part,
                             hipStream_t s);
hipError_t launch_round_node(const RoundNode* nodes, int n_nodes, const RoundDesc* ds, double* err, hipStream_t s);
hipError_t launch_round_plan(const RoundDesc* d, const RoundDesc* o, double inv_s, int s_is_a, double* out,
                             size_t total, hipStream_t s);

// ---- warm-start data movement (defined in gmot_mlp.hip) ----
// One star instance: center node 0 (free), edges (0, l) for leaves l = 1..L in
// that order, all supports of size n.  Potentials of edge l-1 sit at
// base + 2n(l-1): Lam_(0,l) (n values) then Lam_(l,0) (n values).
struct StarDesc {
  const double* lg_leaf;     // log mu of leaves 1..L, concatenated [L * n]
  double* lam0;              // slot-0 base (written by the warm start)
  const double* lam_cur;     // base of the slot holding the committed leaf potentials
};
hipError_t launch_star_features(const StarDesc* stars, int count, int L, int n, float shift, float scale, float* x,
                                hipStream_t s);
hipError_t launch_star_targets(const StarDesc* stars, int count, int L, int n, float out_scale, float* t,
                               hipStream_t s);
hipError_t launch_star_apply(const StarDesc* stars, int count, int L, int n, const float* y, float out_scale,
                             int* rejected, hipStream_t s);

}  // namespace gmot

#ifdef __cplusplus
#include <atomic>
#include <map>
// Host-side context shared by the runtime and the MLP host code.
// Node-kernel block shape: W waves per block, R rows per lane, H lane groups per
// wave (tiles of 64 * R / H rows: 32, 64 or 128).
struct NodeShape {
  int W, R, H;
  int G = 1;  // 1: the uniform-grid kernels (k_msg_grid, k_sep_horner) where a problem admits them
};

struct gmot_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  double clk_hz = 1.0e8;
  std::map<uint64_t, NodeShape> tuned;  // instance shapes key -> tuned node-kernel shape
  void* scratch = nullptr;                         // small tables of the warm-start calls
  size_t scratch_size = 0;
  // a second stream and two events, used only while capturing graphs: kernel
  // groups of one node stage that touch different instances are captured as
  // parallel branches (fork on ev_fork, join on ev_join)
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // One reference for the caller of gmot_ctx_create and one per live problem,
  // batch and network: the context is freed when the last one is dropped, so
  // the objects may be destroyed in any order.
  std::atomic<int> refs{1};
};
void gmot_ctx_retain(gmot_ctx* ctx);
void gmot_ctx_release(gmot_ctx* ctx);
#include <string>
// Sets the message gmot_last_error reports for the calling thread.
void gmot_set_last_error(const std::string& msg);
// Accessors of the network object for the runtime's warm-start entry point.
struct gmot_mlp;
int gmot_mlp_widths(const gmot_mlp* m, int* n_in, int* n_out);
int gmot_mlp_workspace(gmot_mlp* m, int B, float** x, float** y);
#endif
