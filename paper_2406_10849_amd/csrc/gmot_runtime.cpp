// Host runtime of libgmot: validation, device arenas, work lists, the
// graph-captured half-sweep loop and the FP64 evaluation pass.
//
// Schedule (Algorithm tree_local_reg): the tree is 2-coloured by BFS from node
// 0; class 0 ("S1", the class of node 0 unless the caller picks the other one)
// is updated on odd half-sweeps, class 1 on even ones.  A half-sweep is two
// launches: the message kernel over every (row tile, column split) of every
// message into the class, then the node kernel over the class's nodes.  `k`
// half-sweeps are captured in one hipGraph; the host replays it two deep and
// polls a pinned 4-byte counter of finished instances between replays.  Once an
// instance has stopped, its kernels return at entry, so overshooting replays
// cost only empty launches.
#include "gmot.h"
#include "gmot_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <array>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

using namespace gmot;

namespace {

thread_local std::string g_last_error;
struct TileStats { int rows = 0, max_splits = 0, blocks[2] = {0, 0}; };
thread_local TileStats g_tiles;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

}  // namespace

// The message gmot_last_error reports, also set by the network's entry points.
void gmot_set_last_error(const std::string& msg) { g_last_error = msg; }

namespace {

#define HIPCHK(x)                                                                     \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) return fail(GMOT_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct Plan;
struct RoundState;


struct gmot_problem {
  gmot_ctx* ctx = nullptr;
  int N = 0, E = 0, dim = 1, cost_kind = 0, first_color = 0;
  double eps = 1.0;
  std::vector<int> sizes, edges;
  std::vector<uint8_t> fixed;
  std::vector<std::vector<int>> nbrs;      // ascending
  std::vector<std::vector<int>> nbr_de;    // directed edge id of (j, nbrs[j][i])
  std::vector<int> colour;                 // 0 = first class
  std::vector<int64_t> node_off;           // [N+1] point offsets
  std::vector<int64_t> de_off;             // [2E+1]; de 2e = (a,b), 2e+1 = (b,a)
  std::vector<int64_t> cost_off;           // [E+1] offsets of C_e; C_e^T follows all C_e
  int64_t total_pts = 0, total_de = 0, total_cost = 0;
  void* arena = nullptr;
  double* d_support = nullptr;
  double* d_lg = nullptr;
  double* d_mu = nullptr;
  double* d_lam[kSlots] = {};
  double* d_mfull = nullptr;
  double* d_abar = nullptr;
  double* d_qbar = nullptr;
  double* d_c = nullptr;  // [kSlots N]: node normaliser c_j, slot s at kSlots j + s (0 for constrained nodes)
  float* d_cost = nullptr;
  float* d_cost_tile = nullptr;           // per directed edge, tile-major (node kernel)
  std::vector<int64_t> tcost_off;         // [2E + 1] offsets into d_cost_tile
  // separable messages: every support is a row-major grid (D = 2, on-the-fly
  // squared-Euclidean cost); grid_cols[j] = points per grid row of node j
  bool sep = false;
  std::vector<int> grid_cols;
  // messages from uniform one-dimensional grids (k_msg_grid): every support is
  // y_j = y_0 + j h to within a few ulps, and every message keeps the powers of
  // its rows' ratios within 2^(+-kGridRange)
  bool grid = false;
  int grid_rows_lane = 1;  // rows per lane the grid kernel may take (1, or 2 when 128-row spans qualify)
  // separable messages whose grid coordinate lists are all uniform and whose
  // passes keep the powers of each output's ratio within 2^(+-kGridRange):
  // k_sep_horner instead of k_sep_pass
  bool sep_h = false;
  int grid_rows(int j) const { return (int)((sizes[j] + grid_cols[j] - 1) / grid_cols[j]); }
  int64_t t = 1;
  uint64_t version = 0;   // bumped whenever the held state changes
  Plan* plan = nullptr;
  RoundState* round = nullptr;

  const double* c_ptr(int j) const { return fixed[j] ? nullptr : d_c + kSlots * j; }

  int de_of(int j, int k) const {
    for (size_t i = 0; i < nbrs[j].size(); ++i)
      if (nbrs[j][i] == k) return nbr_de[j][i];
    return -1;
  }
  // slot holding the committed value of class c's potentials
  int slot_of_class(int c) const { return c == 0 ? (int)((t / 2) % kSlots) : (int)(((t - 1) / 2) % kSlots); }
};

// Tile group of separable instances (after the explicit-cost and D = 1..3 groups).
constexpr int kSepGroup = 4;
// Tile group of instances on uniform one-dimensional grids (k_msg_grid + k_node_sep).
constexpr int kGridGroup = 5;
// Tile group of separable instances on uniform grids (k_sep_horner + k_node_sep).
constexpr int kSepHGroup = 6;
// Rows per node-stage tile of separable instances.
constexpr int kSepTileRows = 64;
// In a class whose k_node groups have fewer than kSplitBelowTiles tiles, nodes
// of degree >= kSplitDeg take their messages as one message-only item per
// (tile, edge) and their update in k_node_sep, so a few large high-degree
// nodes still fill the device (in a large batch the extra blocks and launch
// cost more than they save).  GMOT_SPLIT_DEG=d splits every node of degree >= d.
constexpr int kSplitDeg = 4;
constexpr int64_t kSplitBelowTiles = 2048;
// Blocks per launch a separable pass aims at when its messages are few.
constexpr int64_t kSepTargetBlocks = 2048;

// Timing mode: events per half-sweep, and back-to-back repeats of the message
// stage between the first two (so their mean excludes the event overhead).
// Kernel groups of a node stage: explicit cost, D = 1, 2, 3 (k_node), separable
// grids (k_sep_pass + k_node_sep), uniform one-dimensional grids (k_msg_grid +
// k_node_sep), separable uniform grids (k_sep_horner + k_node_sep).
constexpr int kGroups = 7;
constexpr int kStepEvents = 4 + 2 * kGroups;
constexpr int kMsgBurst = 4;

// A captured run of k half-sweeps.  The timed variant is not captured: it
// launches the k half-sweeps directly, recording one of two alternating chains
// of kStepEvents * k events (see Plan::launch_tstep), so one chain can be read
// back while the next replay runs.
struct GraphEntry {
  bool fp64 = false, timed = false, per_node = false, fused = false;
  int start = 0, k = 0;
  uint64_t lists = 0;  // key of the work lists it was captured on (Plan::list_key)
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  std::vector<hipEvent_t> ev[2];
};

struct Plan {
  gmot_ctx* ctx = nullptr;
  std::vector<gmot_problem*> probs;
  int W = 4;                 // waves per node-kernel block
  int NR = 1;                // node-kernel rows per lane
  int NH = 1;                // node-kernel lane groups per wave (tiles of 64 * NR / NH rows)
  int R = 1;                 // evaluation message kernel: rows per lane
  int target_blocks = 1024;  // evaluation message kernel: blocks per class (via column splits)
  std::vector<MsgDesc> msgs;
  std::vector<K1Item> items[2][4];  // [class][0 = explicit, 1..3 = dim]
  std::vector<std::pair<int, int>> msg_items[2][4];  // per message: (first item, item count)
  std::vector<std::pair<int, int>> msg_item_range;    // per plan message: (first item, count) in its (class, group)
  // items of the messages the node kernel's groups evaluate come first; the
  // uniform-grid groups' messages (after them) are evaluated by their own kernels
  int items_general[2][4] = {};
  std::vector<NodeItem> nodes[2];
  std::vector<InstState> inst;
  int total_nodes = 0;
  void* arena = nullptr;
  MsgDesc* d_msgs = nullptr;
  K1Item* d_items[2][4] = {};
  NodeItem* d_nodes[2] = {};
  InstState* d_inst = nullptr;
  double4* d_node_eval = nullptr;
  int* d_ndone = nullptr;
  double2* d_partial = nullptr;
  double* d_wmax = nullptr;
  double* d_tpart = nullptr;
  // node-kernel tiles per [class][0 = explicit, 1..3 = dim, kSepGroup = separable
  // grids, kGridGroup = uniform one-dimensional grids (message items, one per
  // (edge, 64 rows))]
  std::vector<TileItem> tiles[2][kGroups];
  std::vector<std::pair<int, int>> node_tiles[2][kGroups];  // per node: (first tile, tile count)
  TileItem* d_tiles[2][kGroups] = {};
  // Nodes of degree >= split_deg in the k_node groups: their tiles above are
  // message-only items, one per (tile, edge), and their update runs in
  // k_node_sep over these 64-row tiles (per node: (first, count), count 0 for
  // the other nodes, in node_tiles order).  The grid group's nodes all update
  // here (index kSepGroup is unused).
  int split_deg = 0;
  int grid_R = 1;  // rows per lane of the grid group's message items (64 grid_R rows each)
  std::vector<TileItem> upd_tiles[2][kGroups];
  std::vector<std::pair<int, int>> node_upd[2][kGroups];
  TileItem* d_upd_tiles[2][kGroups] = {};
  // separable instances: items of both passes per class, and per node of the
  // separable group (in node_tiles[c][kSepGroup] order) its (first, count) in each
  std::vector<SepItem> sep_items[2], sep_items2[2];
  std::vector<std::array<int, 4>> node_sep[2];
  SepItem* d_sep_items[2] = {};
  SepItem* d_sep_items2[2] = {};
  // separable instances on uniform grids: tasks of both passes per class
  // ([class][pass]), and per node of the separable group its (first, count) in each
  std::vector<SepTask> sep_tasks[2][2];
  std::vector<std::array<int, 4>> node_sept[2];
  SepTask* d_sep_tasks[2][2] = {};
  size_t sep_lds[2][2] = {};  // dynamic LDS bytes per block, [class][pass]
  double* d_sepT = nullptr;
  int* d_inst_slot = nullptr;  // evaluation pass: committed slot of each class, per instance
  double4* d_msg_eval = nullptr;  // evaluation pass: per-message sums of the plans' marginals
  // per instance: whether the uniform-grid kernels (k_msg_grid, k_sep_horner)
  // sum its messages, and the plan message of each directed edge (its
  // destination node's side)
  std::vector<uint8_t> inst_horner;
  std::vector<std::vector<int>> de_msg;
  int rec_rows = 64;         // rows per tile record
  int* h_ndone = nullptr;  // pinned, two mailboxes
  std::vector<GraphEntry> graphs;
  // Work lists of the node stage for a subset of the instances.  The fields
  // above hold the lists in use (key list_key; 0 = every instance); the sets
  // here hold the others, each in its own device buffer, so that a graph
  // captured on a set stays valid while another is in use.  Once most
  // instances of a batch have stopped, run_plan swaps in the lists of the
  // running ones, so its launches no longer start blocks that only find their
  // instance stopped.
  struct ListSet {
    uint64_t key = 0;
    void* buf = nullptr;
    std::vector<TileItem> tiles[2][kGroups], upd[2][kGroups];
    std::vector<SepItem> sep[2], sep2[2];
    std::vector<SepTask> sept[2][2];
    TileItem* d_tiles[2][kGroups] = {};
    TileItem* d_upd[2][kGroups] = {};
    SepItem* d_sep[2] = {};
    SepItem* d_sep2[2] = {};
    SepTask* d_sept[2][2] = {};
  };
  std::vector<ListSet> list_sets;
  uint64_t list_key = 0;
  // evaluation pair pass: edge descriptors, work items and partial sums (kept
  // between calls; the descriptors are rewritten each call)
  void* pair_buf = nullptr;
  size_t pair_buf_size = 0;

  void swap_lists(ListSet& L) {
    for (int c = 0; c < 2; ++c) {
      for (int g = 0; g < kGroups; ++g) {
        std::swap(tiles[c][g], L.tiles[c][g]);
        std::swap(d_tiles[c][g], L.d_tiles[c][g]);
      }
      for (int g = 0; g < kGroups; ++g) {
        std::swap(upd_tiles[c][g], L.upd[c][g]);
        std::swap(d_upd_tiles[c][g], L.d_upd[c][g]);
      }
      std::swap(sep_items[c], L.sep[c]);
      std::swap(sep_items2[c], L.sep2[c]);
      std::swap(d_sep_items[c], L.d_sep[c]);
      std::swap(d_sep_items2[c], L.d_sep2[c]);
      for (int q = 0; q < 2; ++q) {
        std::swap(sep_tasks[c][q], L.sept[c][q]);
        std::swap(d_sep_tasks[c][q], L.d_sept[c][q]);
      }
    }
    std::swap(list_key, L.key);
    std::swap(buf_in_use, L.buf);
  }
  void* buf_in_use = nullptr;  // device buffer of the lists in use (nullptr: the plan arena)
  // Put the lists of `key` in use; false when no set has that key.
  bool select_lists(uint64_t key) {
    if (key == list_key) return true;
    for (auto& L : list_sets)
      if (L.key == key) {
        swap_lists(L);
        return true;
      }
    return false;
  }
  TileStats stats;
  std::vector<double> inst_pairs[2];  // (x, y) pairs of each instance's messages into class c
  std::vector<double> inst_group_pairs[2][kGroups];  // the same per kernel group
  gmot_stats acc{};

  ~Plan() {
    for (auto& g : graphs)
      for (int i = 0; i < 2; ++i) {
        if (g.exec[i]) (void)hipGraphExecDestroy(g.exec[i]);
        for (hipEvent_t e : g.ev[i]) (void)hipEventDestroy(e);
      }
    for (auto& L : list_sets)
      if (L.buf) (void)hipFree(L.buf);
    if (buf_in_use) (void)hipFree(buf_in_use);
    if (pair_buf) (void)hipFree(pair_buf);
    if (arena) (void)hipFree(arena);
    if (h_ndone) (void)hipHostFree(h_ndone);
  }

  Tables tables(int c, int dk) const {
    Tables tb{};
    tb.msgs = d_msgs;
    tb.items = dk >= 0 && dk < 4 ? d_items[c][dk] : nullptr;
    tb.nodes = d_nodes[c];
    tb.inst = d_inst;
    tb.node_eval = d_node_eval;
    tb.ndone = d_ndone;
    tb.tiles = dk >= 0 ? d_tiles[c][dk] : nullptr;
    tb.colour = c;
    tb.sep_items = d_sep_items[c];
    tb.sep_items2 = d_sep_items2[c];
    tb.sep_tasks = d_sep_tasks[c][0];
    tb.sep_tasks2 = d_sep_tasks[c][1];
    tb.rec_rows = rec_rows;
    tb.inst_slot = d_inst_slot;
    tb.msg_eval = d_msg_eval;
    return tb;
  }

  // Kernel group g (0 = explicit cost, 1..3 = dimension, kSepGroup =
  // separable grids, kGridGroup = uniform one-dimensional grids) of the node
  // stage of class c: one launch (three for the separable group, two for the
  // grid group), or with per_node one per node (the same tiles, issued node
  // by node).  *fin_pending: the first launch also carries the finalise
  // step of the other class's half-sweep (the previous launch's), one block
  // per instance.
  hipError_t launch_group(int c, int g, bool fp64, hipStream_t s, bool per_node, bool* fin_pending) const {
    hipError_t e = hipSuccess;
    if (g < kSepGroup) {
      if (tiles[c][g].empty()) return hipSuccess;
      if (!per_node) {
        Tables tb = tables(c, g);
        if (*fin_pending) {
          tb.n_fin = (int)inst.size();
          tb.fin_colour = 1 - c;
          tb.fin_nodes = d_nodes[1 - c];
          *fin_pending = false;
        }
        if ((e = launch_node(tb, (int)tiles[c][g].size(), g, W, NR, NH, fp64, s)) != hipSuccess) return e;
        if (upd_tiles[c][g].empty()) return hipSuccess;
        tb = tables(c, g);
        tb.tiles = d_upd_tiles[c][g];
        return launch_node_sep(tb, (int)upd_tiles[c][g].size(), s);
      }
      for (size_t i = 0; i < node_tiles[c][g].size(); ++i) {
        Tables tb = tables(c, g);
        tb.tiles += node_tiles[c][g][i].first;
        if ((e = launch_node(tb, node_tiles[c][g][i].second, g, W, NR, NH, fp64, s)) != hipSuccess) return e;
        if (node_upd[c][g][i].second > 0) {
          tb = tables(c, g);
          tb.tiles = d_upd_tiles[c][g] + node_upd[c][g][i].first;
          if ((e = launch_node_sep(tb, node_upd[c][g][i].second, s)) != hipSuccess) return e;
        }
      }
      return hipSuccess;
    }
    if (g == kGridGroup) {
      // uniform one-dimensional grids: the messages, then the node stage
      if (tiles[c][g].empty()) return hipSuccess;
      if (!per_node) {
        Tables tb = tables(c, g);
        if (*fin_pending) {
          tb.n_fin = (int)inst.size();
          tb.fin_colour = 1 - c;
          tb.fin_nodes = d_nodes[1 - c];
          *fin_pending = false;
        }
        if ((e = launch_msg_grid(tb, (int)tiles[c][g].size(), grid_R, false, s)) != hipSuccess) return e;
        tb = tables(c, g);
        tb.tiles = d_upd_tiles[c][g];
        return launch_node_sep(tb, (int)upd_tiles[c][g].size(), s);
      }
      for (size_t i = 0; i < node_tiles[c][g].size(); ++i) {
        Tables tb = tables(c, g);
        tb.tiles += node_tiles[c][g][i].first;
        if ((e = launch_msg_grid(tb, node_tiles[c][g][i].second, grid_R, false, s)) != hipSuccess) return e;
        tb = tables(c, g);
        tb.tiles = d_upd_tiles[c][g] + node_upd[c][g][i].first;
        if ((e = launch_node_sep(tb, node_upd[c][g][i].second, s)) != hipSuccess) return e;
      }
      return hipSuccess;
    }
    if (g == kSepHGroup) {
      // separable instances on uniform grids: both passes by Horner's rule,
      // then the node stage
      if (sep_tasks[c][0].empty()) return hipSuccess;
      if (!per_node) {
        Tables tb = tables(c, g);
        if (*fin_pending) {
          tb.n_fin = (int)inst.size();
          tb.fin_colour = 1 - c;
          tb.fin_nodes = d_nodes[1 - c];
          *fin_pending = false;
        }
        if ((e = launch_sep_horner(tb, 0, (int)sep_tasks[c][0].size(), false, s)) != hipSuccess) return e;
        tb.n_fin = 0;
        if ((e = launch_sep_horner(tb, 1, (int)sep_tasks[c][1].size(), false, s)) != hipSuccess) return e;
        return launch_node_sep(tb, (int)tiles[c][g].size(), s);
      }
      for (size_t i = 0; i < node_sept[c].size(); ++i) {
        Tables tb = tables(c, g);
        tb.sep_tasks += node_sept[c][i][0];
        tb.sep_tasks2 += node_sept[c][i][2];
        if ((e = launch_sep_horner(tb, 0, node_sept[c][i][1], false, s)) != hipSuccess) return e;
        if ((e = launch_sep_horner(tb, 1, node_sept[c][i][3], false, s)) != hipSuccess) return e;
        tb.tiles += node_tiles[c][g][i].first;
        if ((e = launch_node_sep(tb, node_tiles[c][g][i].second, s)) != hipSuccess) return e;
      }
      return hipSuccess;
    }
    // separable instances: the two passes of their messages, then the node stage
    if (sep_items[c].empty()) return hipSuccess;
    if (!per_node) {
      Tables tb = tables(c, kSepGroup);
      if (*fin_pending) {
        tb.n_fin = (int)inst.size();
        tb.fin_colour = 1 - c;
        tb.fin_nodes = d_nodes[1 - c];
        *fin_pending = false;
      }
      if ((e = launch_sep_pass(tb, 0, (int)sep_items[c].size(), sep_lds[c][0], fp64, s)) != hipSuccess) return e;
      tb.n_fin = 0;
      if ((e = launch_sep_pass(tb, 1, (int)sep_items2[c].size(), sep_lds[c][1], fp64, s)) != hipSuccess) return e;
      return launch_node_sep(tb, (int)tiles[c][kSepGroup].size(), s);
    }
    for (size_t i = 0; i < node_sep[c].size(); ++i) {
      Tables tb = tables(c, kSepGroup);
      tb.sep_items += node_sep[c][i][0];
      tb.sep_items2 += node_sep[c][i][2];
      if ((e = launch_sep_pass(tb, 0, node_sep[c][i][1], sep_lds[c][0], fp64, s)) != hipSuccess) return e;
      if ((e = launch_sep_pass(tb, 1, node_sep[c][i][3], sep_lds[c][1], fp64, s)) != hipSuccess) return e;
      tb.tiles += node_tiles[c][kSepGroup][i].first;
      if ((e = launch_node_sep(tb, node_tiles[c][kSepGroup][i].second, s)) != hipSuccess) return e;
    }
    return hipSuccess;
  }

  bool group_empty(int c, int g) const {
    return g == kSepGroup ? sep_items[c].empty() : g == kSepHGroup ? sep_tasks[c][0].empty() : tiles[c][g].empty();
  }
  static bool aux_group(int g) { return g == kSepGroup || g == kSepHGroup; }

  // The node stage of class c: every kernel group in turn.  With fused, the
  // first launch also carries the finalise step of the previous half-sweep.
  hipError_t launch_node_stage(int c, bool fp64, hipStream_t s, bool per_node, bool fused = false) const {
    bool fin_pending = fused;
    for (int g = 0; g < kGroups; ++g) {
      const hipError_t e = launch_group(c, g, fp64, s, per_node, &fin_pending);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }

  // The fused node stage under graph capture: the other groups on s and the
  // separable groups on the context's second stream as parallel branches
  // (they work on different instances), joined before the stage ends; the
  // finalise blocks ride in the first launch on s.  Groups on one side only:
  // launch_node_stage.
  hipError_t launch_node_stage_forked(int c, bool fp64, hipStream_t s) const {
    bool d_any = false, a_any = false;
    for (int g = 0; g < kGroups; ++g) (aux_group(g) ? a_any : d_any) |= !group_empty(c, g);
    if (!d_any || !a_any) return launch_node_stage(c, fp64, s, false, true);
    hipError_t e;
    bool fin_d = true, fin_sep = false;
    if ((e = hipEventRecord(ctx->ev_fork, s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(ctx->aux, ctx->ev_fork, 0)) != hipSuccess) return e;
    for (int g = 0; g < kGroups; ++g)
      if (aux_group(g) && (e = launch_group(c, g, fp64, ctx->aux, false, &fin_sep)) != hipSuccess) return e;
    for (int g = 0; g < kGroups; ++g)
      if (!aux_group(g) && (e = launch_group(c, g, fp64, s, false, &fin_d)) != hipSuccess) return e;
    if ((e = hipEventRecord(ctx->ev_join, ctx->aux)) != hipSuccess) return e;
    return hipStreamWaitEvent(s, ctx->ev_join, 0);
  }

  // One half-sweep of class c: the node stage, then the finalise kernel.  With
  // events (timing mode, direct launches): ev[0], the node stage kMsgBurst
  // times, ev[1]; then per kernel group g ev[4 + 2g], the group kMsgBurst
  // times, ev[5 + 2g]; then the node stage, ev[2], the finalise kernel, ev[3].
  // A repeat of the node stage or of a group reads the same state and
  // rewrites the same slots (only its shifts differ), so a burst's mean is the
  // duration without the event overhead.
  // Fused (no events, layer schedule): the node stage alone, its first launch
  // finalising the previous half-sweep.
  hipError_t launch_tstep(int c, bool fp64, hipStream_t s, const hipEvent_t* ev = nullptr,
                          bool per_node = false, bool fused = false, bool forked = false) const {
    hipError_t e;
    if (fused) return forked ? launch_node_stage_forked(c, fp64, s) : launch_node_stage(c, fp64, s, false, true);
    if (ev) {
      if ((e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
      for (int r = 0; r < kMsgBurst; ++r)
        if ((e = launch_node_stage(c, fp64, s, per_node)) != hipSuccess) return e;
      if ((e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
      for (int g = 0; g < kGroups; ++g) {
        if ((e = hipEventRecord(ev[4 + 2 * g], s)) != hipSuccess) return e;
        for (int r = 0; r < kMsgBurst; ++r) {
          bool no_fin = false;
          if ((e = launch_group(c, g, fp64, s, per_node, &no_fin)) != hipSuccess) return e;
        }
        if ((e = hipEventRecord(ev[5 + 2 * g], s)) != hipSuccess) return e;
      }
    }
    if ((e = launch_node_stage(c, fp64, s, per_node)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
    e = launch_finalize(tables(c, -1), (int)inst.size(), s);
    if (e != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[3], s)) != hipSuccess) return e;
    return hipSuccess;
  }
};

// ---------------------------------------------------------------------------
// plan construction
// ---------------------------------------------------------------------------
static int build_plan(gmot_ctx* ctx, const std::vector<gmot_problem*>& probs, NodeShape shape, Plan** out) {
  std::unique_ptr<Plan> pl(new Plan());
  pl->ctx = ctx;
  pl->probs = probs;
  // explicit-cost tiles keep one row per lane and one lane group (each lane
  // holds its rows' cost chunk in registers)
  for (const gmot_problem* p : probs)
    if (p->cost_kind == GMOT_COST_EXPLICIT) shape.R = shape.H = 1;
  pl->W = shape.W;
  pl->NR = shape.R;
  pl->NH = shape.H;
  pl->split_deg = kSplitDeg;
  // two rows per lane in the grid kernel when every grid instance admits
  // 128-row spans; GMOT_GRID_ROWS=1 keeps one
  // the uniform-grid kernels where a problem admits them, unless the shape
  // turns them off (the autotuner times both)
  const bool use_grid = shape.G != 0;
  auto on_grid = [&](const gmot_problem* p) { return use_grid && p->grid; };
  auto on_sep_h = [&](const gmot_problem* p) { return use_grid && p->sep_h; };
  pl->grid_R = 2;
  for (const gmot_problem* p : probs)
    if (on_grid(p) && p->grid_rows_lane < 2) pl->grid_R = 1;
  if (const char* v = std::getenv("GMOT_GRID_ROWS"))
    if (std::atoi(v) == 1) pl->grid_R = 1;
  bool split_forced = false;
  if (const char* v = std::getenv("GMOT_SPLIT_DEG")) {
    pl->split_deg = std::max(1, std::atoi(v));
    split_forced = true;
  }
  const int TRows = kNodeRowsLane * shape.R / shape.H;
  const int R = pl->R, target_blocks = pl->target_blocks;
  const int TM = 256 * R;
  // node tiles per (class, dimension group), with each node's work (pairs) for ordering
  struct NodeTiles { int node_item, n_tiles, inst; double work; };
  std::vector<NodeTiles> ntl[2][kGroups];

  // messages and node items (class-major within each instance)
  std::vector<int> msg_class;
  std::map<size_t, std::pair<int, int>> msg_src;            // message -> (instance, source node)
  std::map<std::pair<int, int>, std::pair<int, int>> item_of;  // (instance, node) -> (class, node item)
  int err_counter = 0;
  pl->inst_horner.assign(probs.size(), 0);
  pl->de_msg.assign(probs.size(), {});
  for (size_t i = 0; i < probs.size(); ++i) {
    gmot_problem* p = probs[i];
    pl->inst_horner[i] = on_grid(p) || on_sep_h(p) ? 1 : 0;
    pl->de_msg[i].assign(2 * (size_t)p->E, -1);
    InstState st{};
    for (int c = 0; c < 2; ++c) {
      st.node0[c] = (int)pl->nodes[c].size();
      int cnt = 0;
      for (int j = 0; j < p->N; ++j) {
        if (p->colour[j] != c || p->nbrs[j].empty()) continue;
        NodeItem nd{};
        nd.inst = (int)i;
        nd.node = j;
        nd.n = p->sizes[j];
        nd.deg = (int)p->nbrs[j].size();
        nd.fixed = p->fixed[j];
        nd.msg0 = (int)pl->msgs.size();
        nd.err_idx = err_counter++;
        nd.lg = p->d_lg + p->node_off[j];
        nd.mu = p->fixed[j] ? p->d_mu + p->node_off[j] : nullptr;
        nd.abar = p->d_abar + p->node_off[j];
        nd.qbar = p->d_qbar + p->node_off[j];
        nd.c = p->fixed[j] ? nullptr : p->d_c + kSlots * j;
        nd.tiles = (int)ceil_div(p->sizes[j], std::min(TRows, 64));  // tile records: one per 64 rows (32 for 32-row tiles)
        if (p->sep) {
          // terms of the node's messages (both passes)
          double work = 0.0;
          for (int k : p->nbrs[j])
            work += (double)p->grid_rows(k) * p->grid_cols[j] * p->grid_cols[k] +
                    (double)p->sizes[j] * p->grid_rows(k);
          ntl[c][on_sep_h(p) ? kSepHGroup : kSepGroup].push_back(
              {(int)pl->nodes[c].size(), (int)ceil_div(p->sizes[j], kSepTileRows), (int)i, work});
        } else if (on_grid(p)) {
          double src_cols = 0.0;
          for (int k : p->nbrs[j]) src_cols += p->sizes[k];
          ntl[c][kGridGroup].push_back({(int)pl->nodes[c].size(), (int)ceil_div(p->sizes[j], 64), (int)i, src_cols});
        } else {
          double src_cols = 0.0;
          for (int k : p->nbrs[j]) src_cols += p->sizes[k];
          const int dk = p->cost_kind == GMOT_COST_EXPLICIT ? 0 : p->dim;
          ntl[c][dk].push_back({(int)pl->nodes[c].size(), (int)ceil_div(p->sizes[j], TRows), (int)i, src_cols});
        }
        item_of[{(int)i, j}] = {c, (int)pl->nodes[c].size()};
        pl->nodes[c].push_back(nd);
        ++cnt;
        for (size_t q = 0; q < p->nbrs[j].size(); ++q) {
          const int k = p->nbrs[j][q];
          const int de_dst = p->nbr_de[j][q];  // (j,k)
          const int de_src = de_dst ^ 1;       // (k,j)
          MsgDesc md{};
          md.supp_dst = p->d_support + p->node_off[j] * p->dim;
          md.supp_src = p->d_support + p->node_off[k] * p->dim;
          for (int s = 0; s < kSlots; ++s) {
            md.lam_src[s] = p->d_lam[s] + p->de_off[de_src];
            md.lam_dst[s] = p->d_lam[s] + p->de_off[de_dst];
          }
          md.lg_src = p->d_lg + p->node_off[k];
          md.c_src = p->c_ptr(k);
          md.mfull = p->d_mfull + p->de_off[de_dst];
          if (p->cost_kind == GMOT_COST_EXPLICIT) {
            const int e = de_dst >> 1;
            // stored src-major: dst = b uses C_e (rows a = src), dst = a uses C_e^T
            const bool dst_is_b = (de_dst & 1) == 1;
            md.cost = dst_is_b ? p->d_cost + p->cost_off[e] : p->d_cost + p->total_cost + p->cost_off[e];
            md.cost_tile = p->d_cost_tile + p->tcost_off[de_dst];
          }
          md.n_dst = p->sizes[j];
          md.n_src = p->sizes[k];
          md.src_free = p->fixed[k] ? 0 : 1;
          if (p->sep) {
            md.rows_src = p->grid_rows(k);
            md.cols_src = p->grid_cols[k];
            md.rows_dst = p->grid_rows(j);
            md.cols_dst = p->grid_cols[j];
          }
          msg_src[pl->msgs.size()] = {(int)i, k};
          md.inst = (int)i;
          md.dim = p->dim;
          md.cost_kind = p->cost_kind;
          md.eps = p->eps;
          md.grid = on_grid(p) || on_sep_h(p) ? 1 : 0;
          pl->de_msg[i][de_dst] = (int)pl->msgs.size();
          pl->msgs.push_back(md);
          msg_class.push_back(c);
        }
      }
      st.nnodes[c] = cnt;
    }
    pl->inst.push_back(st);
  }
  pl->total_nodes = err_counter;
  for (int c = 0; c < 2; ++c) {
    pl->inst_pairs[c].assign(probs.size(), 0.0);
    for (int g = 0; g < kGroups; ++g) pl->inst_group_pairs[c][g].assign(probs.size(), 0.0);
  }
  // (x, y) term evaluations of the node stage: n_j n_k per message, or
  // A_k B_j B_k + n_j A_k for a separable one (its two passes)
  for (size_t m = 0; m < pl->msgs.size(); ++m) {
    const MsgDesc& md = pl->msgs[m];
    const double ev = probs[md.inst]->sep
                          ? (double)md.rows_src * md.cols_dst * md.cols_src + (double)md.n_dst * md.rows_src
                          : (double)md.n_dst * md.n_src;
    pl->inst_pairs[msg_class[m]][md.inst] += ev;
    const int grp = probs[md.inst]->sep       ? (on_sep_h(probs[md.inst]) ? kSepHGroup : kSepGroup)
                    : on_grid(probs[md.inst]) ? kGridGroup
                    : md.cost_kind == GMOT_COST_EXPLICIT ? 0
                                                         : md.dim;
    pl->inst_group_pairs[msg_class[m]][grp][md.inst] += ev;
  }

  // column splits: enough blocks per class to fill the device
  int64_t row_tiles[2] = {0, 0};
  for (size_t m = 0; m < pl->msgs.size(); ++m) row_tiles[msg_class[m]] += ceil_div(pl->msgs[m].n_dst, TM);
  int64_t want_ns[2];
  for (int c = 0; c < 2; ++c)
    want_ns[c] = row_tiles[c] > 0 ? std::max<int64_t>(1, (target_blocks + row_tiles[c] / 2) / row_tiles[c]) : 1;
  int64_t partial_total = 0;
  std::vector<int64_t> partial_off(pl->msgs.size());
  pl->stats = TileStats();
  pl->msg_item_range.assign(pl->msgs.size(), {0, 0});
  auto horner = [&](size_t m) { return on_grid(probs[pl->msgs[m].inst]) || on_sep_h(probs[pl->msgs[m].inst]); };
  std::vector<size_t> order;
  for (size_t m = 0; m < pl->msgs.size(); ++m)
    if (!horner(m)) order.push_back(m);
  const size_t n_general = order.size();
  for (size_t m = 0; m < pl->msgs.size(); ++m)
    if (horner(m)) order.push_back(m);
  for (size_t oi = 0; oi < order.size(); ++oi) {
    const size_t m = order[oi];
    if (oi == n_general)
      for (int c = 0; c < 2; ++c)
        for (int dk = 0; dk < 4; ++dk) pl->items_general[c][dk] = (int)pl->items[c][dk].size();
    MsgDesc& md = pl->msgs[m];
    const int c = msg_class[m];
    int64_t ns = std::min<int64_t>(want_ns[c], std::max<int64_t>(1, ceil_div(md.n_src, 64)));
    const int64_t cw = ceil_div(md.n_src, ns);
    ns = ceil_div(md.n_src, cw);
    md.ns = (int)ns;
    partial_off[m] = partial_total;
    partial_total += ns * md.n_dst;
    const int dk = md.cost_kind == GMOT_COST_EXPLICIT ? 0 : md.dim;
    pl->msg_items[c][dk].push_back({(int)pl->items[c][dk].size(), (int)(ceil_div(md.n_dst, TM) * ns)});
    pl->msg_item_range[m] = pl->msg_items[c][dk].back();
    for (int64_t rt = 0; rt < ceil_div(md.n_dst, TM); ++rt)
      for (int64_t s = 0; s < ns; ++s) {
        K1Item it{};
        it.msg = (int)m;
        it.row0 = (int)(rt * TM);
        it.col0 = (int)(s * cw);
        it.ncols = (int)std::min<int64_t>(cw, md.n_src - s * cw);
        it.split = (int)s;
        it.inst = md.inst;
        pl->items[c][dk].push_back(it);
      }
  }
  if (n_general == order.size())
    for (int c = 0; c < 2; ++c)
      for (int dk = 0; dk < 4; ++dk) pl->items_general[c][dk] = (int)pl->items[c][dk].size();
  // Separable passes: a block takes as many lines of one message as fit
  // kSepStage staged values and kSepMaxOut outputs (at least one line: grid
  // sides are at most kSepMaxSide), with dynamic LDS for the largest block.
  // Fewer lines per block when a class has few lines in all (large messages):
  // about kSepTargetBlocks blocks per launch, but at least one output per thread.
  int64_t sep_total_lines[2][2] = {{0, 0}, {0, 0}};
  for (int c = 0; c < 2; ++c)
    for (const NodeTiles& q : ntl[c][kSepGroup]) {
      const NodeItem& qn = pl->nodes[c][q.node_item];
      for (int m = qn.msg0; m < qn.msg0 + qn.deg; ++m) {
        sep_total_lines[c][0] += pl->msgs[m].rows_src;
        sep_total_lines[c][1] += pl->msgs[m].cols_dst;
      }
    }
  auto sep_geom = [&](const MsgDesc& md, int c, int pass, int* lines, int* per) {
    const int outs = pass == 0 ? md.cols_dst : md.rows_dst, inner = pass == 0 ? md.cols_src : md.rows_src;
    *lines = pass == 0 ? md.rows_src : md.cols_dst;
    const int cap = std::max(1, std::min({*lines, kSepStage / sep_row_stride(inner), kSepMaxOut / outs}));
    const int64_t want = std::max<int64_t>(ceil_div(sep_total_lines[c][pass], kSepTargetBlocks),
                                           ceil_div(64 * kSepWaves, outs));
    *per = (int)std::min<int64_t>(cap, want);
    return (size_t)sizeof(double) * ((size_t)*per * sep_row_stride(inner) + sep_inner_even(inner));
  };
  // node-kernel tiles: the heaviest nodes (most source columns per row) first,
  // so their long blocks start early; each node's tiles stay consecutive
  bool split_class[2];
  for (int c = 0; c < 2; ++c) {
    int64_t class_tiles = 0;
    for (int dk = 0; dk < kSepGroup; ++dk)
      for (const NodeTiles& q : ntl[c][dk]) class_tiles += q.n_tiles;
    split_class[c] = split_forced || class_tiles < kSplitBelowTiles;
  }
  for (int c = 0; c < 2; ++c)
    for (int dk = 0; dk < kGroups; ++dk) {
      std::stable_sort(ntl[c][dk].begin(), ntl[c][dk].end(),
                       [](const NodeTiles& u, const NodeTiles& v) { return u.work > v.work; });
      const int rows = dk == kSepGroup || dk == kSepHGroup ? kSepTileRows : TRows;
      for (const NodeTiles& q : ntl[c][dk]) {
        const NodeItem& qn = pl->nodes[c][q.node_item];
        if (dk == kGridGroup) {
          // one message item per (edge, 64 grid_R rows), the rows of one edge
          // together (their waves share the source's columns), then the
          // update's 64-row tiles
          const int mt = (int)ceil_div(qn.n, 64 * pl->grid_R);
          pl->node_tiles[c][dk].push_back({(int)pl->tiles[c][dk].size(), mt * qn.deg});
          for (int k = 0; k < qn.deg; ++k)
            for (int r = 0; r < mt; ++r)
              pl->tiles[c][dk].push_back({q.node_item, r * 64 * pl->grid_R, q.inst, qn.msg0 + k, 1, qn.n, qn.fixed, 1});
          pl->node_upd[c][dk].push_back({(int)pl->upd_tiles[c][dk].size(), q.n_tiles});
          for (int r = 0; r < q.n_tiles; ++r)
            pl->upd_tiles[c][dk].push_back({q.node_item, r * 64, q.inst, qn.msg0, qn.deg, qn.n, qn.fixed, 0});
          continue;
        }
        const bool split = dk < kSepGroup && split_class[c] && qn.deg >= pl->split_deg;
        pl->node_tiles[c][dk].push_back({(int)pl->tiles[c][dk].size(), q.n_tiles * (split ? qn.deg : 1)});
        if (split) {
          // one message-only item per (tile, edge), then the update's 64-row tiles
          for (int r = 0; r < q.n_tiles; ++r)
            for (int k = 0; k < qn.deg; ++k)
              pl->tiles[c][dk].push_back({q.node_item, r * rows, q.inst, qn.msg0 + k, 1, qn.n, qn.fixed, 1});
          const int nu = (int)ceil_div(qn.n, 64);
          pl->node_upd[c][dk].push_back({(int)pl->upd_tiles[c][dk].size(), nu});
          for (int r = 0; r < nu; ++r)
            pl->upd_tiles[c][dk].push_back({q.node_item, r * 64, q.inst, qn.msg0, qn.deg, qn.n, qn.fixed, 0});
        } else {
          for (int r = 0; r < q.n_tiles; ++r)
            pl->tiles[c][dk].push_back({q.node_item, r * rows, q.inst, qn.msg0, qn.deg, qn.n, qn.fixed, 0});
          if (dk < kSepGroup) pl->node_upd[c][dk].push_back({(int)pl->upd_tiles[c][dk].size(), 0});
        }
        if (dk == kSepGroup) {
          std::array<int, 4> r{(int)pl->sep_items[c].size(), 0, (int)pl->sep_items2[c].size(), 0};
          for (int m = qn.msg0; m < qn.msg0 + qn.deg; ++m)
            for (int pass = 0; pass < 2; ++pass) {
              int lines = 0, per = 0;
              const size_t lds = sep_geom(pl->msgs[m], c, pass, &lines, &per);
              pl->sep_lds[c][pass] = std::max(pl->sep_lds[c][pass], lds);
              auto& items = pass == 0 ? pl->sep_items[c] : pl->sep_items2[c];
              for (int l0 = 0; l0 < lines; l0 += per) items.push_back({m, l0, q.inst, std::min(per, lines - l0)});
            }
          r[1] = (int)pl->sep_items[c].size() - r[0];
          r[3] = (int)pl->sep_items2[c].size() - r[2];
          pl->node_sep[c].push_back(r);
        }
        if (dk == kSepHGroup) {
          // one wave per (64 outputs, kSepTaskLines lines) of each message and pass
          std::array<int, 4> r{(int)pl->sep_tasks[c][0].size(), 0, (int)pl->sep_tasks[c][1].size(), 0};
          for (int m = qn.msg0; m < qn.msg0 + qn.deg; ++m)
            for (int pass = 0; pass < 2; ++pass) {
              const MsgDesc& md = pl->msgs[m];
              const int lines = pass == 0 ? md.rows_src : md.cols_dst, outs = pass == 0 ? md.cols_dst : md.rows_dst;
              auto& tk = pl->sep_tasks[c][pass];
              for (int o0 = 0; o0 < outs; o0 += 64)
                for (int l = 0; l < lines; l += kSepTaskLines) tk.push_back({m, l, o0, q.inst});
            }
          r[1] = (int)pl->sep_tasks[c][0].size() - r[0];
          r[3] = (int)pl->sep_tasks[c][1].size() - r[2];
          pl->node_sept[c].push_back(r);
        }
      }
    }
  pl->rec_rows = std::min(TRows, 64);
  // first-pass sums (then their shifts) of separable messages
  int64_t sepT_total = 0;
  std::vector<int64_t> sepT_off(pl->msgs.size(), -1);
  for (size_t m = 0; m < pl->msgs.size(); ++m)
    if (probs[pl->msgs[m].inst]->sep) {
      sepT_off[m] = sepT_total;
      sepT_total += (int64_t)pl->msgs[m].rows_src * pl->msgs[m].cols_dst;
    }
  int64_t wmax_total = 0;
  std::vector<int64_t> wmax_off(pl->msgs.size());
  for (size_t m = 0; m < pl->msgs.size(); ++m) {
    wmax_off[m] = wmax_total;
    wmax_total += (int64_t)pl->msgs[m].n_dst * kMaxRanges;
  }
  // tile records of every node
  int64_t tpart_total = 0;
  std::vector<int64_t> tpart_off[2];
  for (int c = 0; c < 2; ++c)
    for (const NodeItem& nd : pl->nodes[c]) {
      tpart_off[c].push_back(tpart_total);
      tpart_total += (int64_t)nd.tiles * (nd.deg + kRecExtra);
    }
  pl->stats.rows = TRows;
  pl->stats.max_splits = shape.W;
  for (int c = 0; c < 2; ++c) {
    pl->stats.blocks[c] = 0;
    for (int dk = 0; dk < kGroups; ++dk) pl->stats.blocks[c] += (int)pl->tiles[c][dk].size();
    for (int dk = 0; dk < kGroups; ++dk) pl->stats.blocks[c] += (int)pl->upd_tiles[c][dk].size();
  }

  // one device allocation for every table
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = align_up(off, 256);
    off = o + std::max<size_t>(bytes, 1);
    return o;
  };
  const size_t o_msgs = take(sizeof(MsgDesc) * pl->msgs.size());
  size_t o_items[2][4];
  for (int c = 0; c < 2; ++c)
    for (int dk = 0; dk < 4; ++dk) o_items[c][dk] = take(sizeof(K1Item) * pl->items[c][dk].size());
  size_t o_nodes[2];
  for (int c = 0; c < 2; ++c) o_nodes[c] = take(sizeof(NodeItem) * pl->nodes[c].size());
  const size_t o_inst = take(sizeof(InstState) * pl->inst.size());
  const size_t o_eval = take(sizeof(double4) * std::max(1, pl->total_nodes));
  const size_t o_ndone = take(sizeof(int) * 4);
  const size_t o_part = take(sizeof(double2) * std::max<int64_t>(1, partial_total));
  const size_t o_wmax = take(sizeof(double) * std::max<int64_t>(1, wmax_total));
  size_t o_tiles[2][kGroups];
  for (int c = 0; c < 2; ++c)
    for (int dk = 0; dk < kGroups; ++dk) o_tiles[c][dk] = take(sizeof(TileItem) * pl->tiles[c][dk].size());
  size_t o_upd[2][kGroups];
  for (int c = 0; c < 2; ++c)
    for (int dk = 0; dk < kGroups; ++dk) o_upd[c][dk] = take(sizeof(TileItem) * pl->upd_tiles[c][dk].size());
  const size_t o_tpart = take(sizeof(double) * std::max<int64_t>(1, tpart_total));
  size_t o_sep[2], o_sep2[2];
  for (int c = 0; c < 2; ++c) o_sep[c] = take(sizeof(SepItem) * pl->sep_items[c].size());
  for (int c = 0; c < 2; ++c) o_sep2[c] = take(sizeof(SepItem) * pl->sep_items2[c].size());
  size_t o_sept[2][2];
  for (int c = 0; c < 2; ++c)
    for (int q = 0; q < 2; ++q) o_sept[c][q] = take(sizeof(SepTask) * pl->sep_tasks[c][q].size());
  const size_t o_sepT = take(sizeof(double) * 2 * std::max<int64_t>(1, sepT_total));
  const size_t o_islot = take(sizeof(int) * 2 * probs.size());
  const size_t o_meval = take(sizeof(double4) * std::max<size_t>(1, pl->msgs.size()));
  const size_t total = off;
  if (hipMalloc(&pl->arena, total) != hipSuccess) return fail(GMOT_ENOMEM, "plan arena allocation failed");
  char* base = (char*)pl->arena;
  pl->d_msgs = (MsgDesc*)(base + o_msgs);
  for (int c = 0; c < 2; ++c)
    for (int dk = 0; dk < 4; ++dk) pl->d_items[c][dk] = (K1Item*)(base + o_items[c][dk]);
  for (int c = 0; c < 2; ++c) pl->d_nodes[c] = (NodeItem*)(base + o_nodes[c]);
  pl->d_inst = (InstState*)(base + o_inst);
  pl->d_node_eval = (double4*)(base + o_eval);
  pl->d_ndone = (int*)(base + o_ndone);
  pl->d_partial = (double2*)(base + o_part);
  pl->d_wmax = (double*)(base + o_wmax);
  for (int c = 0; c < 2; ++c)
    for (int dk = 0; dk < kGroups; ++dk) pl->d_tiles[c][dk] = (TileItem*)(base + o_tiles[c][dk]);
  for (int c = 0; c < 2; ++c)
    for (int dk = 0; dk < kGroups; ++dk) pl->d_upd_tiles[c][dk] = (TileItem*)(base + o_upd[c][dk]);
  pl->d_tpart = (double*)(base + o_tpart);
  for (int c = 0; c < 2; ++c) pl->d_sep_items[c] = (SepItem*)(base + o_sep[c]);
  for (int c = 0; c < 2; ++c) pl->d_sep_items2[c] = (SepItem*)(base + o_sep2[c]);
  for (int c = 0; c < 2; ++c)
    for (int q = 0; q < 2; ++q) pl->d_sep_tasks[c][q] = (SepTask*)(base + o_sept[c][q]);
  pl->d_sepT = (double*)(base + o_sepT);
  pl->d_inst_slot = (int*)(base + o_islot);
  pl->d_msg_eval = (double4*)(base + o_meval);
  for (int c = 0; c < 2; ++c)
    for (size_t i = 0; i < pl->nodes[c].size(); ++i) pl->nodes[c][i].tpart = pl->d_tpart + tpart_off[c][i];
  for (size_t m = 0; m < pl->msgs.size(); ++m) {
    pl->msgs[m].partial = pl->d_partial + partial_off[m];
    pl->msgs[m].wmax = pl->d_wmax + wmax_off[m];
    pl->msgs[m].sepT = sepT_off[m] >= 0 ? pl->d_sepT + sepT_off[m] : nullptr;
    pl->msgs[m].sepM = sepT_off[m] >= 0 ? pl->d_sepT + std::max<int64_t>(1, sepT_total) + sepT_off[m] : nullptr;
    // the source node's records (constrained sources too: read, then ignored)
    const auto src = item_of.at(msg_src.at(m));
    const NodeItem& sn = pl->nodes[src.first][src.second];
    pl->msgs[m].src_tpart = sn.tpart;
    pl->msgs[m].src_tiles = sn.tiles;
    pl->msgs[m].src_deg = sn.deg;
  }

  hipStream_t s = ctx->stream;
  HIPCHK(hipMemcpyAsync(pl->d_msgs, pl->msgs.data(), sizeof(MsgDesc) * pl->msgs.size(), hipMemcpyHostToDevice, s));
  for (int c = 0; c < 2; ++c) {
    for (int dk = 0; dk < 4; ++dk)
      if (!pl->items[c][dk].empty())
        HIPCHK(hipMemcpyAsync(pl->d_items[c][dk], pl->items[c][dk].data(), sizeof(K1Item) * pl->items[c][dk].size(),
                              hipMemcpyHostToDevice, s));
    if (!pl->nodes[c].empty())
      HIPCHK(hipMemcpyAsync(pl->d_nodes[c], pl->nodes[c].data(), sizeof(NodeItem) * pl->nodes[c].size(),
                            hipMemcpyHostToDevice, s));
    for (int dk = 0; dk < kGroups; ++dk)
      if (!pl->tiles[c][dk].empty())
        HIPCHK(hipMemcpyAsync(pl->d_tiles[c][dk], pl->tiles[c][dk].data(),
                              sizeof(TileItem) * pl->tiles[c][dk].size(), hipMemcpyHostToDevice, s));
    for (int dk = 0; dk < kGroups; ++dk)
      if (!pl->upd_tiles[c][dk].empty())
        HIPCHK(hipMemcpyAsync(pl->d_upd_tiles[c][dk], pl->upd_tiles[c][dk].data(),
                              sizeof(TileItem) * pl->upd_tiles[c][dk].size(), hipMemcpyHostToDevice, s));
    if (!pl->sep_items[c].empty())
      HIPCHK(hipMemcpyAsync(pl->d_sep_items[c], pl->sep_items[c].data(), sizeof(SepItem) * pl->sep_items[c].size(),
                            hipMemcpyHostToDevice, s));
    if (!pl->sep_items2[c].empty())
      HIPCHK(hipMemcpyAsync(pl->d_sep_items2[c], pl->sep_items2[c].data(),
                            sizeof(SepItem) * pl->sep_items2[c].size(), hipMemcpyHostToDevice, s));
    for (int q = 0; q < 2; ++q)
      if (!pl->sep_tasks[c][q].empty())
        HIPCHK(hipMemcpyAsync(pl->d_sep_tasks[c][q], pl->sep_tasks[c][q].data(),
                              sizeof(SepTask) * pl->sep_tasks[c][q].size(), hipMemcpyHostToDevice, s));
  }
  // one-pass shifts start at 0; the first two half-sweeps of every call take two passes anyway
  HIPCHK(hipMemsetAsync(pl->d_wmax, 0, sizeof(double) * std::max<int64_t>(1, wmax_total), s));
  HIPCHK(hipMemsetAsync(pl->d_sepT, 0, sizeof(double) * 2 * std::max<int64_t>(1, sepT_total), s));
  HIPCHK(hipHostMalloc((void**)&pl->h_ndone, sizeof(int) * 2, hipHostMallocDefault));
  HIPCHK(hipStreamSynchronize(s));
  g_tiles = pl->stats;
  *out = pl.release();
  return GMOT_OK;
}

static uint64_t shape_key(const std::vector<gmot_problem*>& probs) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a
  auto mix = [&](uint64_t v) {
    h ^= v;
    h *= 1099511628211ull;
  };
  mix(probs.size());
  for (const gmot_problem* p : probs) {
    mix((uint64_t)p->N);
    mix((uint64_t)p->dim);
    mix((uint64_t)p->cost_kind);
    mix((uint64_t)p->first_color);
    for (int s : p->sizes) mix((uint64_t)s);
    for (int e : p->edges) mix((uint64_t)e);
  }
  return h;
}

constexpr NodeShape kDefaultShape{4, 2, 1};

static bool valid_shape(const NodeShape& s) {
  return (s.W == 2 || s.W == 4 || s.W == 8 || s.W == 16) && (s.R == 1 || s.R == 2) && (s.H == 1 || s.H == 2);
}

// Without a tuned choice, the uniform-grid kernels serve a plan whose node
// stage gives them at least kGridMinWaves message waves (one per SIMD of the
// device); a smaller plan fills the device better through the node kernel's
// column ranges (a single star, the 32-node chain).
constexpr int64_t kGridMinWaves = 1024;

static int grid_default(const std::vector<gmot_problem*>& probs) {
  int64_t waves = 0;  // both classes' message waves, halved below
  for (const gmot_problem* p : probs) {
    if (!p->grid && !p->sep_h) continue;
    for (int e = 0; e < p->E; ++e)
      for (int d = 0; d < 2; ++d) {
        const int k = p->edges[2 * e + d], j = p->edges[2 * e + 1 - d];  // message k -> j
        if (p->grid) {
          waves += ceil_div(p->sizes[j], 64 * p->grid_rows_lane);
        } else {
          const int rows_k = p->grid_rows(k), cols_j = p->grid_cols[j];
          waves += ceil_div(rows_k, kSepTaskLines) * ceil_div(cols_j, 64) +
                   ceil_div(cols_j, kSepTaskLines) * ceil_div(p->grid_rows(j), 64);
        }
      }
  }
  return waves / 2 >= kGridMinWaves ? 1 : 0;
}

// Node-kernel block shape: a tuned choice cached in the context for these
// shapes, else the default (with the uniform-grid kernels as grid_default
// decides); GMOT_NODE_SHAPE="W,R" or "W,R,H" (W in 2, 4, 8, 16; R in 1, 2; H
// in 1, 2) overrides the block shape and GMOT_GRID=0 or 1 the grid kernels.
static NodeShape choose_shape(gmot_ctx* ctx, const std::vector<gmot_problem*>& probs) {
  NodeShape sh = kDefaultShape;
  auto it = ctx->tuned.find(shape_key(probs));
  if (it != ctx->tuned.end()) sh = it->second;
  else sh.G = grid_default(probs);
  if (const char* v = std::getenv("GMOT_NODE_SHAPE")) {
    NodeShape e{0, 0, 1, sh.G};
    const int got = std::sscanf(v, "%d,%d,%d", &e.W, &e.R, &e.H);
    if (got >= 2 && valid_shape(e)) sh = e;
  }
  if (const char* v = std::getenv("GMOT_GRID")) sh.G = std::atoi(v) != 0 ? 1 : 0;
  return sh;
}

static int capture_one(Plan* pl, bool fp64, bool per_node, bool fused, int start, int k,
                       const std::vector<hipEvent_t>* ev, hipGraphExec_t* out) {
  hipStream_t s = pl->ctx->stream;
  HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int i = 0; i < k && le == hipSuccess; ++i)
    le = pl->launch_tstep((start + i) & 1, fp64, s, ev ? ev->data() + kStepEvents * i : nullptr, per_node, fused,
                          !ev && !per_node);
  hipGraph_t graph = nullptr;
  hipError_t ce = hipStreamEndCapture(s, &graph);
  if (le != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(GMOT_EDEVICE, std::string("kernel launch during capture: ") + hipGetErrorString(le));
  }
  if (ce != hipSuccess) return fail(GMOT_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
  hipGraphExec_t exec = nullptr;
  hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return fail(GMOT_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
  *out = exec;
  return GMOT_OK;
}

static int get_graph(Plan* pl, bool fp64, bool per_node, bool fused, int start, int k, bool timed,
                     GraphEntry** out) {
  for (auto& g : pl->graphs)
    if (g.fp64 == fp64 && g.per_node == per_node && g.fused == fused && g.start == start && g.k == k &&
        g.timed == timed && g.lists == pl->list_key) {
      *out = &g;
      return GMOT_OK;
    }
  GraphEntry g;
  g.fp64 = fp64;
  g.start = start;
  g.k = k;
  g.lists = pl->list_key;
  g.timed = timed;
  g.per_node = per_node;
  g.fused = fused;
  if (timed) {
    // HIP events recorded by graph nodes cannot be timed, so the timed variant
    // launches directly on the stream with two alternating event chains.
    for (int c = 0; c < 2; ++c) {
      g.ev[c].resize(kStepEvents * k);
      for (auto& e : g.ev[c]) HIPCHK(hipEventCreate(&e));
    }
  } else {
    int rc = capture_one(pl, fp64, per_node, fused, start, k, nullptr, &g.exec[0]);
    if (rc) return rc;
  }
  pl->graphs.push_back(std::move(g));
  *out = &pl->graphs.back();
  return GMOT_OK;
}

// Batches of at least kCompactMin instances swap in the work lists of their
// running instances whenever these number at most 1/kCompactRatio of the
// instances in the lists in use; at most kMaxListSets compacted sets (and
// their graphs) are kept.
constexpr int kCompactMin = 64;
constexpr int kCompactRatio = 2;
constexpr size_t kMaxListSets = 8;

// Puts in use the work lists of the instances with running[i] != 0 (taken, in
// order, from the lists in use, which hold them all), from the stored set with
// that instance set's key or a new one in a device buffer of its own.
static int compact_lists(Plan* pl, const std::vector<char>& running, int* count) {
  uint64_t key = 1469598103934665603ull;  // FNV-1a over the running instance indexes
  int cnt = 0;
  for (size_t i = 0; i < running.size(); ++i)
    if (running[i]) {
      key = (key ^ (uint64_t)i) * 1099511628211ull;
      ++cnt;
    }
  key |= 1;  // 0 stands for every instance
  *count = cnt;
  if (pl->select_lists(key)) return GMOT_OK;
  if (pl->list_sets.size() >= kMaxListSets) {
    // drop the stored compacted sets and the graphs captured on them
    for (auto it = pl->graphs.begin(); it != pl->graphs.end();) {
      const bool stale = it->lists != 0 && it->lists != pl->list_key;
      if (stale) {
        for (int i = 0; i < 2; ++i) {
          if (it->exec[i]) (void)hipGraphExecDestroy(it->exec[i]);
          for (hipEvent_t e : it->ev[i]) (void)hipEventDestroy(e);
        }
        it = pl->graphs.erase(it);
      } else {
        ++it;
      }
    }
    for (auto it = pl->list_sets.begin(); it != pl->list_sets.end();) {
      if (it->key != 0) {
        if (it->buf) (void)hipFree(it->buf);
        it = pl->list_sets.erase(it);
      } else {
        ++it;
      }
    }
  }
  Plan::ListSet L;
  L.key = key;
  auto keep = [&](int inst) { return inst >= 0 && inst < (int)running.size() && running[inst]; };
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = align_up(off, 256);
    off = o + std::max<size_t>(bytes, 1);
    return o;
  };
  size_t o_t[2][kGroups], o_u[2][kGroups], o_s[2], o_s2[2], o_k[2][2];
  for (int c = 0; c < 2; ++c) {
    for (int g = 0; g < kGroups; ++g) {
      for (const TileItem& t : pl->tiles[c][g])
        if (keep(t.inst)) L.tiles[c][g].push_back(t);
      o_t[c][g] = take(sizeof(TileItem) * L.tiles[c][g].size());
    }
    for (int g = 0; g < kGroups; ++g) {
      for (const TileItem& t : pl->upd_tiles[c][g])
        if (keep(t.inst)) L.upd[c][g].push_back(t);
      o_u[c][g] = take(sizeof(TileItem) * L.upd[c][g].size());
    }
    for (const SepItem& it : pl->sep_items[c])
      if (keep(it.inst)) L.sep[c].push_back(it);
    for (const SepItem& it : pl->sep_items2[c])
      if (keep(it.inst)) L.sep2[c].push_back(it);
    o_s[c] = take(sizeof(SepItem) * L.sep[c].size());
    o_s2[c] = take(sizeof(SepItem) * L.sep2[c].size());
    for (int q = 0; q < 2; ++q) {
      for (const SepTask& tk : pl->sep_tasks[c][q])
        if (keep(tk.inst)) L.sept[c][q].push_back(tk);
      o_k[c][q] = take(sizeof(SepTask) * L.sept[c][q].size());
    }
  }
  if (hipMalloc(&L.buf, off) != hipSuccess) return fail(GMOT_ENOMEM, "compacted work lists");
  char* b = (char*)L.buf;
  hipStream_t s = pl->ctx->stream;
  for (int c = 0; c < 2; ++c) {
    for (int g = 0; g < kGroups; ++g) {
      L.d_tiles[c][g] = (TileItem*)(b + o_t[c][g]);
      if (!L.tiles[c][g].empty())
        HIPCHK(hipMemcpyAsync(L.d_tiles[c][g], L.tiles[c][g].data(), sizeof(TileItem) * L.tiles[c][g].size(),
                              hipMemcpyHostToDevice, s));
    }
    for (int g = 0; g < kGroups; ++g) {
      L.d_upd[c][g] = (TileItem*)(b + o_u[c][g]);
      if (!L.upd[c][g].empty())
        HIPCHK(hipMemcpyAsync(L.d_upd[c][g], L.upd[c][g].data(), sizeof(TileItem) * L.upd[c][g].size(),
                              hipMemcpyHostToDevice, s));
    }
    L.d_sep[c] = (SepItem*)(b + o_s[c]);
    L.d_sep2[c] = (SepItem*)(b + o_s2[c]);
    if (!L.sep[c].empty())
      HIPCHK(hipMemcpyAsync(L.d_sep[c], L.sep[c].data(), sizeof(SepItem) * L.sep[c].size(), hipMemcpyHostToDevice, s));
    if (!L.sep2[c].empty())
      HIPCHK(hipMemcpyAsync(L.d_sep2[c], L.sep2[c].data(), sizeof(SepItem) * L.sep2[c].size(),
                            hipMemcpyHostToDevice, s));
    for (int q = 0; q < 2; ++q) {
      L.d_sept[c][q] = (SepTask*)(b + o_k[c][q]);
      if (!L.sept[c][q].empty())
        HIPCHK(hipMemcpyAsync(L.d_sept[c][q], L.sept[c][q].data(), sizeof(SepTask) * L.sept[c][q].size(),
                              hipMemcpyHostToDevice, s));
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  pl->list_sets.push_back(std::move(L));
  pl->swap_lists(pl->list_sets.back());
  return GMOT_OK;
}

// Run every instance of the plan from its problem's held state.
// Instances with active[i] == 0 do not run and keep their result untouched.
// The stop test applies from half-sweep max(2, t_start + min_updates) on: the
// paper's loop never stops before the second half-sweep, and the FP64 verify
// phase must first make one class exact in FP64.
static int run_plan(Plan* pl, const gmot_opts* o, gmot_result* outs, const std::vector<char>* active = nullptr,
                    int64_t min_updates = 0, int64_t stall_window = 0, std::vector<char>* stalled = nullptr) {
  hipStream_t s = pl->ctx->stream;
  const size_t n = pl->probs.size();
  int parity = -1;
  bool mixed = false;
  int already = 0;
  for (size_t i = 0; i < n; ++i) {
    gmot_problem* p = pl->probs[i];
    InstState& st = pl->inst[i];
    st.vdone[0] = st.vdone[1] = 1;
    if (active && !(*active)[i]) {
      st.t = p->t;
      st.done = kMaxSteps;
      st.updates = 0;
      ++already;
      continue;
    }
    st.t = p->t;
    st.t_first = p->t;
    st.min_check_t = std::max<int64_t>(2, p->t + min_updates);
    st.updates = 0;
    st.max_updates = o->max_steps;
    st.tol = o->tol;
    st.err_sum = INFINITY;
    st.err_max = INFINITY;
    st.checked_t = 0;
    st.counter = 0;
    st.clk_start = st.clk_stop = 0;
    // by default the first computation of every message in this call takes two passes
    st.onepass_from = o->msg_passes == GMOT_PASSES_TWO ? INT64_MAX
                      : o->msg_passes == GMOT_PASSES_ONE ? p->t
                                                          : p->t + 2;
    st.best_err = INFINITY;
    st.best_t = p->t;
    st.stall_window = stall_window;
    st.done = kRunning;
    if (p->E == 0) {  // single node: nothing to scale
      st.done = kConverged;
      st.err_sum = st.err_max = 0.0;
      ++already;
      continue;
    }
    const int par = (int)(p->t & 1);
    // instances at the other parity sit out one launch and then run in step
    if (parity < 0) parity = par;
    if (par != parity) mixed = true;
  }
  // The finalise step rides in the next half-sweep's node launch unless the
  // half-sweeps are timed, issued node by node, or instances start at both
  // parities.  The fused node blocks of half-sweep t + 1 then run before t is
  // decided; they write only slots that no state the decision keeps uses.
  const bool fused = o->timing == 0 && o->schedule != GMOT_SCHED_PER_NODE && !mixed;
  for (size_t i = 0; i < n; ++i) {
    InstState& st = pl->inst[i];
    if (st.done != kRunning) continue;
    const int c0 = (st.t & 1) ? 0 : 1;  // odd half-sweeps update class 0
    st.vt[c0] = st.t;
    st.vdone[c0] = 0;
    // the other class's first half-sweep: known in advance when fused, else
    // published by the finalise step of this one
    st.vt[1 - c0] = fused ? st.t + 1 : 0;
    st.vdone[1 - c0] = 0;
  }
  HIPCHK(hipMemcpyAsync(pl->d_inst, pl->inst.data(), sizeof(InstState) * n, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(pl->d_ndone, &already, sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  if (already < (int)n) {
    int k = o->check_every > 0 ? o->check_every : 16;
    if (k & 1) ++k;
    if (k > o->max_steps + 1) k = (int)std::max<int64_t>(2, (o->max_steps + 1) & ~int64_t(1));
    const int start = parity == 1 ? 0 : 1;  // odd t updates class 0
    const bool fp64 = o->precision == GMOT_PREC_FP64;
    const bool timed = o->timing != 0;
    const bool per_node = o->schedule == GMOT_SCHED_PER_NODE;
    const bool no_graph = std::getenv("GMOT_NO_GRAPH") != nullptr && !timed;
    // every run starts on the lists of all instances
    if (!pl->select_lists(0)) return fail(GMOT_ESTATE, "the full work lists of the plan are missing");
    // GMOT_COMPACT_RATIO=r compacts at 1/r instead (r >= 2), 0 never
    int compact_ratio = kCompactRatio;
    if (const char* v = std::getenv("GMOT_COMPACT_RATIO")) compact_ratio = std::atoi(v) > 0 ? std::max(2, std::atoi(v)) : 0;
    const bool can_compact = !timed && !no_graph && !per_node && n >= (size_t)kCompactMin && compact_ratio > 0;
    int in_lists = (int)n;  // instances in the lists in use
    int compact_rc = GMOT_OK;
    GraphEntry* g = nullptr;
    if (!no_graph) {
      int rc = get_graph(pl, fp64, per_node, fused, start, k, timed, &g);
      if (rc) return rc;
    }
    HIPCHK(launch_stamp(pl->d_inst, (int)n, s));
    std::vector<int64_t> t_start(n);
    for (size_t i = 0; i < n; ++i) t_start[i] = pl->inst[i].t;
    // every replay advances each running instance by k half-sweeps (one fewer
    // for an instance that starts at the other parity), so this bound is exact;
    // fused, the last half-sweep is decided one launch later
    const int64_t max_launches = ceil_div(o->max_steps + 1, k) + 2;
    hipEvent_t ev[2];
    HIPCHK(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    // per-step durations of timed replays: (step since the start of this call, message ms, node ms)
    struct StepTime { int64_t step; float msg_ms, sweep_ms; float group_ms[kGroups]; };
    std::vector<StepTime> times;
    auto launch_one = [&](int slot) -> hipError_t {
      hipError_t e;
      if (timed) {
        e = hipSuccess;
        for (int i = 0; i < k && e == hipSuccess; ++i)
          e = pl->launch_tstep((start + i) & 1, fp64, s, g->ev[slot].data() + kStepEvents * i, per_node);
      } else if (no_graph) {
        e = hipSuccess;
        for (int i = 0; i < k && e == hipSuccess; ++i)
          e = pl->launch_tstep((start + i) & 1, fp64, s, nullptr, per_node, fused);
      } else {
        e = hipGraphLaunch(g->exec[0], s);
      }
      if (e != hipSuccess) return e;
      e = hipMemcpyAsync(pl->h_ndone + slot, pl->d_ndone, sizeof(int), hipMemcpyDeviceToHost, s);
      if (e != hipSuccess) return e;
      return hipEventRecord(ev[slot], s);
    };
    auto read_times = [&](int64_t replay) -> hipError_t {
      const std::vector<hipEvent_t>& E = g->ev[replay & 1];
      for (int i = 0; i < k; ++i) {
        float a = 0.f, b = 0.f;
        const hipEvent_t* q = E.data() + kStepEvents * i;
        hipError_t e = hipEventElapsedTime(&a, q[0], q[1]);                  // kMsgBurst message stages
        if (e == hipSuccess) e = hipEventElapsedTime(&b, q[1], q[3]);      // groups, one half-sweep
        if (e != hipSuccess) return e;
        StepTime st{replay * k + i, a / kMsgBurst, 0.f, {}};
        const int cls = (start + i) & 1;
        float grp_total = 0.f;
        for (int gi = 0; gi < kGroups && e == hipSuccess; ++gi) {
          float gm = 0.f;
          e = hipEventElapsedTime(&gm, q[4 + 2 * gi], q[5 + 2 * gi]);
          grp_total += gm;
          st.group_ms[gi] = pl->group_empty(cls, gi) ? 0.f : gm / kMsgBurst;
        }
        if (e != hipSuccess) return e;
        st.sweep_ms = b - grp_total;                                         // the half-sweep alone
        times.push_back(st);
      }
      return hipSuccess;
    };
    int64_t launched = 0, waited = 0;
    hipError_t le = hipSuccess;
    while (launched < std::min<int64_t>(2, max_launches) && le == hipSuccess) le = launch_one((int)(launched++ & 1));
    while (le == hipSuccess && waited < launched) {
      const int slot = (int)(waited & 1);
      le = hipEventSynchronize(ev[slot]);
      if (le != hipSuccess) break;
      if (timed) le = read_times(waited);
      if (le != hipSuccess) break;
      ++waited;
      if (pl->h_ndone[slot] >= (int)n) break;
      if (can_compact && (int64_t)((int)n - pl->h_ndone[slot]) * compact_ratio <= in_lists) {
        // drain the replay in flight, then swap in the lists of the running instances
        le = hipStreamSynchronize(s);
        if (le != hipSuccess) break;
        waited = launched;
        if (pl->h_ndone[(launched - 1) & 1] >= (int)n) break;
        std::vector<InstState> now(n);
        le = hipMemcpy(now.data(), pl->d_inst, sizeof(InstState) * n, hipMemcpyDeviceToHost);
        if (le != hipSuccess) break;
        std::vector<char> running(n);
        for (size_t i = 0; i < n; ++i) running[i] = now[i].done == kRunning;
        compact_rc = compact_lists(pl, running, &in_lists);
        if (compact_rc == GMOT_OK) compact_rc = get_graph(pl, fp64, per_node, fused, start, k, timed, &g);
        if (compact_rc != GMOT_OK) break;
        while (le == hipSuccess && launched < max_launches && launched - waited < 2) le = launch_one((int)(launched++ & 1));
        continue;
      }
      if (launched < max_launches) le = launch_one((int)(launched++ & 1));
    }
    hipError_t se = hipStreamSynchronize(s);
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (compact_rc != GMOT_OK) return compact_rc;
    if (le != hipSuccess) return fail(GMOT_EDEVICE, std::string("half-sweep loop: ") + hipGetErrorString(le));
    if (se != hipSuccess) return fail(GMOT_EDEVICE, std::string("half-sweep loop: ") + hipGetErrorString(se));
    pl->acc.graph_launches += launched;
    HIPCHK(hipMemcpy(pl->inst.data(), pl->d_inst, sizeof(InstState) * n, hipMemcpyDeviceToHost));
    if (timed) {
      // last half-sweep (counted from the start of this call) that did work, per instance
      std::vector<int64_t> last(n, -1);
      int64_t last_any = -1;
      for (size_t i = 0; i < n; ++i) {
        const InstState& st = pl->inst[i];
        if (pl->probs[i]->E == 0) continue;
        const int64_t abs_last = (st.done == kConverged || st.done == kStalled) ? st.checked_t
                                 : st.done == kNonFinite ? st.t + 1 : st.t - 1;
        last[i] = abs_last - t_start[i];
        last_any = std::max(last_any, last[i]);
      }
      for (const StepTime& tt : times) {
        if (tt.step > last_any) continue;
        const int c = (int)((start + tt.step) & 1);
        pl->acc.msg_ms += tt.msg_ms;
        pl->acc.sweep_ms += tt.sweep_ms;
        for (int gi = 0; gi < kGroups; ++gi) {
          pl->acc.group_ms[gi] += tt.group_ms[gi];
          for (size_t i = 0; i < n; ++i)
            if (tt.step <= last[i]) pl->acc.group_pairs[gi] += pl->inst_group_pairs[c][gi][i];
        }
        pl->acc.msg_launches += 1;
        for (size_t i = 0; i < n; ++i)
          if (tt.step <= last[i]) pl->acc.msg_pairs += pl->inst_pairs[c][i];
      }
    }
  }
  int rc = GMOT_OK;
  for (size_t i = 0; i < n; ++i) {
    if (active && !(*active)[i]) continue;
    gmot_problem* p = pl->probs[i];
    const InstState& st = pl->inst[i];
    gmot_result& r = outs[i];
    std::memset(&r, 0, sizeof(r));
    if (st.done == kRunning) rc = fail(GMOT_ESTATE, "an instance was still running when the launch budget ended");
    p->t = st.t;
    ++p->version;
    r.status = st.done == kConverged ? GMOT_CONVERGED : st.done == kNonFinite ? GMOT_NONFINITE : GMOT_NOT_CONVERGED;
    if (stalled) (*stalled)[i] = st.done == kStalled;
    r.steps = st.updates;
    r.t = st.t;
    r.err_sum = st.err_sum;
    r.err_max = st.err_max;
    r.seconds = (st.clk_stop > st.clk_start) ? (double)(st.clk_stop - st.clk_start) / pl->ctx->clk_hz : 0.0;
  }
  return rc;
}

// FP32-core solves judge convergence in FP64: the FP32-core loop stops at
// kVerifyMargin * tol, or when its stopping sum has not come 3% below its
// last record for kStallWindow half-sweeps (the FP32 exponentials leave a
// noise floor that can lie above a small tol), and FP64 half-sweeps then run
// from that state
// until the FP64 stopping sum is <= tol, within the remaining step budget.
// On large trees the FP32-core sum can read below the FP64 sum of the same
// state (the iteration settles at the fixed point of the rounded map), which
// the FP64 phase corrects.
constexpr double kVerifyMargin = 0.8;
constexpr int64_t kStallWindow = 64;

static int solve_plan(Plan* pl, const gmot_opts* o, gmot_result* outs) {
  const size_t n = pl->probs.size();
  if (o->precision != GMOT_PREC_FP32CORE || o->skip_verify) return run_plan(pl, o, outs);
  gmot_opts o1 = *o;
  o1.tol = o->tol * kVerifyMargin;
  std::vector<char> stalled(n, 0);
  // tol = 0 asks for exactly max_steps half-sweeps (or an exact fixed point): no stall test
  int rc = run_plan(pl, &o1, outs, nullptr, 0, o->tol > 0.0 ? kStallWindow : 0, &stalled);
  if (rc) return rc;
  std::vector<char> active(n, 0);
  bool any = false;
  int64_t budget = o->max_steps;
  for (size_t i = 0; i < n; ++i) {
    active[i] = (outs[i].status == GMOT_CONVERGED || stalled[i]) && pl->probs[i]->E > 0;
    any = any || active[i];
    if (active[i]) budget = std::min<int64_t>(budget, std::max<int64_t>(1, o->max_steps - outs[i].steps));
  }
  if (!any) return GMOT_OK;
  gmot_opts o2 = *o;
  o2.precision = GMOT_PREC_FP64;
  o2.restart = 0;
  o2.timing = 0;
  o2.check_every = 2;
  o2.max_steps = budget;
  std::vector<gmot_result> r2(n);
  rc = run_plan(pl, &o2, r2.data(), &active, 1);
  if (rc) return rc;
  for (size_t i = 0; i < n; ++i) {
    if (!active[i]) continue;
    outs[i].status = r2[i].status;
    outs[i].steps += r2[i].steps;
    outs[i].t = r2[i].t;
    outs[i].err_sum = r2[i].err_sum;
    outs[i].err_max = r2[i].err_max;
    outs[i].seconds += r2[i].seconds;
  }
  return GMOT_OK;
}

// ---------------------------------------------------------------------------
// problem creation
// ---------------------------------------------------------------------------
static int validate_and_copy(const gmot_tree_desc* d, gmot_problem* p, int first_color) {
  if (!d) return fail(GMOT_EINVAL, "null descriptor");
  if (d->n_nodes < 1) return fail(GMOT_EINVAL, "a tree needs at least one node");
  if (d->n_edges != d->n_nodes - 1) return fail(GMOT_EINVAL, "a tree on N nodes has N-1 edges");
  if (!d->sizes || !d->is_fixed || (d->n_edges > 0 && !d->edges))
    return fail(GMOT_EINVAL, "missing sizes, is_fixed or edges");
  if (!(d->eps > 0.0) || !std::isfinite(d->eps)) return fail(GMOT_EINVAL, "eps must be positive and finite");
  if (d->cost_kind != GMOT_COST_SQEUCLID && d->cost_kind != GMOT_COST_EXPLICIT)
    return fail(GMOT_ENOTSUP, "unknown cost kind");
  if (d->cost_kind == GMOT_COST_SQEUCLID && (d->dim < 1 || d->dim > 3))
    return fail(GMOT_ENOTSUP, "support dimension must be 1, 2 or 3");
  if (d->cost_kind == GMOT_COST_SQEUCLID && !d->support) return fail(GMOT_EINVAL, "missing support points");
  if (d->cost_kind == GMOT_COST_EXPLICIT && d->n_edges > 0 && !d->cost) return fail(GMOT_EINVAL, "missing cost");
  if (first_color < -1 || first_color > 1) return fail(GMOT_EINVAL, "first_color must be -1, 0 or 1");
  const int N = d->n_nodes, E = d->n_edges;
  p->N = N;
  p->E = E;
  p->dim = d->cost_kind == GMOT_COST_SQEUCLID ? d->dim : 1;
  p->cost_kind = d->cost_kind;
  p->eps = d->eps;
  p->sizes.assign(d->sizes, d->sizes + N);
  p->fixed.assign(d->is_fixed, d->is_fixed + N);
  for (int j = 0; j < N; ++j) {
    if (p->sizes[j] < 1) return fail(GMOT_EINVAL, "every node needs at least one support point");
    if (p->sizes[j] > (1 << 24)) return fail(GMOT_ENOTSUP, "support larger than 2^24 points");
    p->fixed[j] = p->fixed[j] ? 1 : 0;
  }
  p->edges.assign(d->edges, d->edges + 2 * E);
  p->nbrs.assign(N, {});
  p->nbr_de.assign(N, {});
  std::vector<std::pair<int, int>> keys;
  for (int e = 0; e < E; ++e) {
    const int a = p->edges[2 * e], b = p->edges[2 * e + 1];
    if (a < 0 || a >= N || b < 0 || b >= N) return fail(GMOT_EINVAL, "edge endpoint out of range");
    if (a == b) return fail(GMOT_EINVAL, "self-loop");
    keys.push_back({std::min(a, b), std::max(a, b)});
  }
  std::sort(keys.begin(), keys.end());
  if (std::adjacent_find(keys.begin(), keys.end()) != keys.end()) return fail(GMOT_EINVAL, "duplicate edge");
  // neighbours in ascending order with their directed-edge ids
  std::vector<std::vector<std::pair<int, int>>> adj(N);
  for (int e = 0; e < E; ++e) {
    const int a = p->edges[2 * e], b = p->edges[2 * e + 1];
    adj[a].push_back({b, 2 * e});
    adj[b].push_back({a, 2 * e + 1});
  }
  for (int j = 0; j < N; ++j) {
    std::sort(adj[j].begin(), adj[j].end());
    for (auto& pr : adj[j]) {
      p->nbrs[j].push_back(pr.first);
      p->nbr_de[j].push_back(pr.second);
    }
  }
  // BFS 2-colouring from node 0; also proves connectivity (with N-1 edges: a tree)
  p->colour.assign(N, -1);
  p->colour[0] = 0;
  std::deque<int> dq{0};
  int seen = 1;
  while (!dq.empty()) {
    const int v = dq.front();
    dq.pop_front();
    for (int w : p->nbrs[v])
      if (p->colour[w] < 0) {
        p->colour[w] = 1 - p->colour[v];
        ++seen;
        dq.push_back(w);
      }
  }
  if (seen != N) return fail(GMOT_EINVAL, "graph is not connected (not a tree)");
  p->first_color = first_color < 0 ? 0 : first_color;
  if (p->first_color == 1)
    for (int j = 0; j < N; ++j) p->colour[j] = 1 - p->colour[j];
  // offsets
  p->node_off.assign(N + 1, 0);
  for (int j = 0; j < N; ++j) p->node_off[j + 1] = p->node_off[j] + p->sizes[j];
  p->total_pts = p->node_off[N];
  p->de_off.assign(2 * E + 1, 0);
  for (int e = 0; e < E; ++e) {
    const int a = p->edges[2 * e], b = p->edges[2 * e + 1];
    p->de_off[2 * e + 1] = p->de_off[2 * e] + p->sizes[a];
    p->de_off[2 * e + 2] = p->de_off[2 * e + 1] + p->sizes[b];
  }
  p->total_de = p->de_off[2 * E];
  p->cost_off.assign(E + 1, 0);
  for (int e = 0; e < E; ++e) {
    const int a = p->edges[2 * e], b = p->edges[2 * e + 1];
    p->cost_off[e + 1] = p->cost_off[e] + (int64_t)p->sizes[a] * p->sizes[b];
  }
  p->total_cost = p->cost_kind == GMOT_COST_EXPLICIT ? p->cost_off[E] : 0;
  // tile-major copies per directed edge de = (j, k): ceil(n_j / 64) * 64 rows x n_k
  p->tcost_off.assign(2 * E + 1, 0);
  for (int de = 0; de < 2 * E; ++de) {
    const int e = de >> 1;
    const int j = (de & 1) ? p->edges[2 * e + 1] : p->edges[2 * e];
    const int k = (de & 1) ? p->edges[2 * e] : p->edges[2 * e + 1];
    const int64_t rows = p->cost_kind == GMOT_COST_EXPLICIT ? ceil_div(p->sizes[j], 64) * 64 : 0;
    p->tcost_off[de + 1] = p->tcost_off[de] + rows * p->sizes[k];
  }
  // marginals
  int64_t nfixed = 0;
  for (int j = 0; j < N; ++j)
    if (p->fixed[j]) nfixed += p->sizes[j];
  if (nfixed > 0 && !d->marginal) return fail(GMOT_EINVAL, "missing marginals");
  {
    int64_t o = 0;
    for (int j = 0; j < N; ++j) {
      if (!p->fixed[j]) continue;
      double sum = 0.0;
      for (int x = 0; x < p->sizes[j]; ++x) {
        const double v = d->marginal[o + x];
        if (!(v >= 0.0) || !std::isfinite(v))
          return fail(GMOT_EMARGINAL, "marginal of node " + std::to_string(j) + " has a negative or non-finite entry");
        sum += v;
      }
      if (std::fabs(sum - 1.0) > 1e-9)
        return fail(GMOT_EMARGINAL, "marginal of node " + std::to_string(j) + " does not sum to 1");
      o += p->sizes[j];
    }
  }
  if (d->cost_kind == GMOT_COST_EXPLICIT) {
    for (int64_t i = 0; i < p->cost_off[E]; ++i)
      if (!std::isfinite(d->cost[i])) return fail(GMOT_EINVAL, "non-finite cost entry");
  }
  return GMOT_OK;
}

static int upload(const gmot_tree_desc* d, gmot_problem* p) {
  hipStream_t s = p->ctx->stream;
  const int64_t P = p->total_pts, D = p->total_de;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = align_up(off, 256);
    off = o + std::max<size_t>(bytes, 1);
    return o;
  };
  const size_t o_sup = take(sizeof(double) * P * p->dim);
  const size_t o_lg = take(sizeof(double) * P);
  const size_t o_mu = take(sizeof(double) * P);
  size_t o_lam[kSlots];
  for (int q = 0; q < kSlots; ++q) o_lam[q] = take(sizeof(double) * D);
  const size_t o_mf = take(sizeof(double) * D);
  const size_t o_ab = take(sizeof(double) * P);
  const size_t o_qb = take(sizeof(double) * P);
  const size_t o_c = take(sizeof(double) * kSlots * p->N);
  const size_t o_cost = take(sizeof(float) * 2 * p->total_cost);
  if (hipMalloc(&p->arena, off) != hipSuccess) return fail(GMOT_ENOMEM, "problem arena allocation failed");
  char* base = (char*)p->arena;
  p->d_support = (double*)(base + o_sup);
  p->d_lg = (double*)(base + o_lg);
  p->d_mu = (double*)(base + o_mu);
  for (int q = 0; q < kSlots; ++q) p->d_lam[q] = (double*)(base + o_lam[q]);
  p->d_mfull = (double*)(base + o_mf);
  p->d_abar = (double*)(base + o_ab);
  p->d_qbar = (double*)(base + o_qb);
  p->d_c = (double*)(base + o_c);
  p->d_cost = p->total_cost ? (float*)(base + o_cost) : nullptr;

  std::vector<double> lg(P, 0.0), mu(P, 0.0), sup((size_t)P * p->dim, 0.0);
  int64_t o = 0;
  for (int j = 0; j < p->N; ++j) {
    if (!p->fixed[j]) continue;
    for (int x = 0; x < p->sizes[j]; ++x) {
      const double v = d->marginal[o + x];
      mu[p->node_off[j] + x] = v;
      lg[p->node_off[j] + x] = v > 0.0 ? std::log(v) : -INFINITY;
    }
    o += p->sizes[j];
  }
  if (d->cost_kind == GMOT_COST_SQEUCLID) std::memcpy(sup.data(), d->support, sizeof(double) * P * p->dim);
  // Separable messages need every support to be a row-major grid: point i of
  // node j equals (first coordinate of point (i / B) B, second coordinate of
  // point i % B) for B = the length of the run of points sharing the first
  // point's first coordinate (the last grid row may be partial).  Exact
  // comparisons: any other layout takes the general message kernel.
  p->grid_cols.assign(p->N, 0);
  p->sep = false;
  if (p->dim == 2 && d->cost_kind == GMOT_COST_SQEUCLID && p->E > 0 && !std::getenv("GMOT_NO_SEP")) {
    bool all = true;
    for (int j = 0; j < p->N && all; ++j) {
      const double* X = sup.data() + p->node_off[j] * 2;
      const int n = p->sizes[j];
      int B = 1;
      while (B < n && X[2 * B] == X[0]) ++B;
      // both grid sides within kSepMaxSide, so a pass block holds at least one line
      all = B <= kSepMaxSide && (n + B - 1) / B <= kSepMaxSide;
      for (int i = 0; i < n && all; ++i)
        all = X[2 * i] == X[2 * (i / B) * B] && X[2 * i + 1] == X[2 * (i % B) + 1];
      p->grid_cols[j] = B;
    }
    p->sep = all;
  }
  // Separable passes by Horner's rule (k_sep_horner): every grid's row and
  // column coordinate lists uniform (as for the one-dimensional grids), and for
  // every message (source k, destination j) and pass, 2 log2e / eps * (half
  // the span of the outputs of a wave) * |h of the inputs| * W <=
  // kGridRange, W the largest power of an output's ratio the pass forms
  // (16 g - 1 for inputs in g <= 4 groups of 16, max(inputs - 1, 64) beyond);
  // the span is that of any 64 consecutive outputs (one wave's).
  p->sep_h = false;
  if (p->sep && !std::getenv("GMOT_NO_GRID")) {
    bool all = true;
    std::vector<double> hR(p->N), hC(p->N), halfR(p->N, 0.0), halfC(p->N, 0.0);
    auto uniform = [](const std::vector<double>& L, double* h) {
      const size_t n = L.size();
      *h = n > 1 ? (L[n - 1] - L[0]) / (double)(n - 1) : 0.0;
      const double tol = 8.0 * DBL_EPSILON * std::max(std::fabs(L[0]), std::fabs(L[n - 1]));
      for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(L[i]) || std::fabs(L[i] - (L[0] + (double)i * *h)) > tol) return false;
      return true;
    };
    auto half64 = [](const std::vector<double>& L) {
      double hs = 0.0;
      for (size_t o0 = 0; o0 < L.size(); o0 += 64) {
        double lo = L[o0], hi = L[o0];
        for (size_t i = o0; i < std::min(L.size(), o0 + 64); ++i) {
          lo = std::min(lo, L[i]);
          hi = std::max(hi, L[i]);
        }
        hs = std::max(hs, 0.5 * (hi - lo));
      }
      return hs;
    };
    for (int j = 0; j < p->N && all; ++j) {
      const double* X = sup.data() + p->node_off[j] * 2;
      const int B = p->grid_cols[j], A = p->grid_rows(j);
      std::vector<double> R(A), Cc(B);
      for (int r = 0; r < A; ++r) R[r] = X[2 * (size_t)r * B];
      for (int c = 0; c < B; ++c) Cc[c] = X[2 * c + 1];
      all = uniform(R, &hR[j]) && uniform(Cc, &hC[j]);
      halfR[j] = half64(R);
      halfC[j] = half64(Cc);
    }
    auto W = [](int inner) { return inner > 64 ? std::max(inner - 1, 64) : 16 * ((inner + 15) / 16) - 1; };
    const double two_kap = 2.0 * kLog2e / p->eps;
    for (int e = 0; e < p->E && all; ++e)
      for (int d = 0; d < 2 && all; ++d) {
        const int k = p->edges[2 * e + d], j = p->edges[2 * e + 1 - d];  // message k -> j
        all = two_kap * halfC[j] * std::fabs(hC[k]) * W(p->grid_cols[k]) <= kGridRange &&
              two_kap * halfR[j] * std::fabs(hR[k]) * W(p->grid_rows(k)) <= kGridRange;
      }
    p->sep_h = all;
  }
  // Messages from uniform one-dimensional grids (k_msg_grid): every support
  // X[i] = X[0] + i h with h = (X[n-1] - X[0]) / (n - 1), to within 8 ulps of
  // its largest magnitude, and for every message (source k, destination j)
  // 2 log2e / eps * (half the span of any 64 rows of j) * |h_k| * max(n_k - 1, 64)
  // <= kGridRange: the kernel forms the powers rho^0 .. rho^64 of a row's
  // ratio, and its sums take rho^j for j < n_k.
  p->grid = false;
  if (p->dim == 1 && d->cost_kind == GMOT_COST_SQEUCLID && p->E > 0 && !std::getenv("GMOT_NO_GRID")) {
    bool all = true;
    std::vector<double> hs(p->N, 0.0), half(p->N, 0.0), half2(p->N, 0.0);
    for (int j = 0; j < p->N && all; ++j) {
      const double* X = sup.data() + p->node_off[j];
      const int n = p->sizes[j];
      const double h = n > 1 ? (X[n - 1] - X[0]) / (double)(n - 1) : 0.0;
      const double tolx = 8.0 * DBL_EPSILON * std::max(std::fabs(X[0]), std::fabs(X[n - 1]));
      for (int i = 0; i < n && all; ++i) all = std::isfinite(X[i]) && std::fabs(X[i] - (X[0] + i * h)) <= tolx;
      hs[j] = h;
      for (int rows = 64; rows <= 128; rows += 64)
        for (int r0 = 0; r0 < n; r0 += rows) {
          double lo = X[r0], hi = X[r0];
          for (int i = r0; i < std::min(n, r0 + rows); ++i) {
            lo = std::min(lo, X[i]);
            hi = std::max(hi, X[i]);
          }
          double& hf = rows == 64 ? half[j] : half2[j];
          hf = std::max(hf, 0.5 * (hi - lo));
        }
    }
    const double two_kap = 2.0 * kLog2e / p->eps;
    bool two = true;  // the same with 128-row spans (two rows per lane)
    for (int e = 0; e < p->E && all; ++e) {
      const int a = p->edges[2 * e], b = p->edges[2 * e + 1];
      const double ga = two_kap * std::fabs(hs[a]) * std::max(p->sizes[a] - 1, 64);  // message a -> b
      const double gb = two_kap * std::fabs(hs[b]) * std::max(p->sizes[b] - 1, 64);  // message b -> a
      all = ga * half[b] <= kGridRange && gb * half[a] <= kGridRange;
      two = two && ga * half2[b] <= kGridRange && gb * half2[a] <= kGridRange;
    }
    p->grid = all;
    p->grid_rows_lane = all && two ? 2 : 1;
  }
  HIPCHK(hipMemcpy(p->d_support, sup.data(), sizeof(double) * P * p->dim, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p->d_lg, lg.data(), sizeof(double) * P, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p->d_mu, mu.data(), sizeof(double) * P, hipMemcpyHostToDevice));
  for (int q = 0; q < kSlots; ++q) HIPCHK(hipMemsetAsync(p->d_lam[q], 0, sizeof(double) * D, s));
  HIPCHK(hipMemsetAsync(p->d_mfull, 0, sizeof(double) * D, s));
  HIPCHK(hipMemsetAsync(p->d_c, 0, sizeof(double) * kSlots * p->N, s));
  if (p->total_cost) {
    HIPCHK(hipMemcpy(p->d_cost, d->cost, sizeof(float) * p->total_cost, hipMemcpyHostToDevice));
    std::vector<float> tr;
    for (int e = 0; e < p->E; ++e) {
      const int a = p->edges[2 * e], b = p->edges[2 * e + 1];
      const int na = p->sizes[a], nb = p->sizes[b];
      tr.assign((size_t)na * nb, 0.0f);
      const float* src = d->cost + p->cost_off[e];
      for (int x = 0; x < na; ++x)
        for (int y = 0; y < nb; ++y) tr[(size_t)y * na + x] = src[(size_t)x * nb + y];
      HIPCHK(hipMemcpy(p->d_cost + p->total_cost + p->cost_off[e], tr.data(), sizeof(float) * tr.size(),
                       hipMemcpyHostToDevice));
    }
    if (hipMalloc(&p->d_cost_tile, sizeof(float) * p->tcost_off[2 * p->E]) != hipSuccess)
      return fail(GMOT_ENOMEM, "tile-major cost allocation failed");
    for (int de = 0; de < 2 * p->E; ++de) {
      const int e = de >> 1;
      const int a = p->edges[2 * e], b = p->edges[2 * e + 1];
      const int na = p->sizes[a], nb = p->sizes[b];
      const bool dst_b = de & 1;
      const int nd = dst_b ? nb : na, ns = dst_b ? na : nb;
      tr.assign((size_t)(p->tcost_off[de + 1] - p->tcost_off[de]), 0.0f);
      const float* src = d->cost + p->cost_off[e];  // C_e row-major: (a, b) at a * nb + b
      for (int x = 0; x < nd; ++x)
        for (int y = 0; y < ns; ++y)
          tr[((size_t)(x >> 6) * ns + y) * 64 + (x & 63)] = dst_b ? src[(size_t)y * nb + x] : src[(size_t)x * nb + y];
      HIPCHK(hipMemcpy(p->d_cost_tile + p->tcost_off[de], tr.data(), sizeof(float) * tr.size(), hipMemcpyHostToDevice));
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  return GMOT_OK;
}

static int ensure_plan(gmot_problem* p) {
  if (p->plan) return GMOT_OK;
  return build_plan(p->ctx, {p}, choose_shape(p->ctx, {p}), &p->plan);
}

// Mean device time of an FP32-core half-sweep (node stage and finalise
// kernel) under this plan: a few real
// half-sweeps from the held state, which is snapshotted before and restored
// after (potential slots, node normalisers and counters).
static int time_plan(Plan* pl, double* ms) {
  hipStream_t s = pl->ctx->stream;
  const size_t n = pl->probs.size();
  std::vector<size_t> off(n + 1, 0);
  for (size_t i = 0; i < n; ++i) {
    const gmot_problem* p = pl->probs[i];
    off[i + 1] = off[i] + kSlots * ((size_t)p->total_de + (size_t)p->N);
  }
  double* snap = nullptr;
  if (hipMalloc(&snap, sizeof(double) * std::max<size_t>(1, off[n])) != hipSuccess)
    return fail(GMOT_ENOMEM, "autotune snapshot");
  std::vector<int64_t> t_saved(n);
  hipError_t e = hipSuccess;
  auto copy_state = [&](bool save) {
    for (size_t i = 0; i < n && e == hipSuccess; ++i) {
      gmot_problem* p = pl->probs[i];
      double* b = snap + off[i];
      const size_t D = p->total_de;
      const hipMemcpyKind k = hipMemcpyDeviceToDevice;
      for (int q = 0; q < kSlots && e == hipSuccess; ++q)
        e = hipMemcpyAsync(save ? b + q * D : p->d_lam[q], save ? p->d_lam[q] : b + q * D, sizeof(double) * D, k, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(save ? b + kSlots * D : p->d_c, save ? p->d_c : b + kSlots * D,
                           sizeof(double) * kSlots * p->N, k, s);
      if (save) t_saved[i] = p->t;
      else p->t = t_saved[i];
    }
  };
  copy_state(true);
  const gmot_stats acc = pl->acc;
  pl->acc = gmot_stats{};
  int rc = GMOT_OK;
  if (e == hipSuccess) {
    gmot_opts o{};
    o.tol = 0.0;
    o.max_steps = 6;
    o.check_every = 2;
    o.precision = GMOT_PREC_FP32CORE;
    o.timing = 1;
    o.skip_verify = 1;
    std::vector<gmot_result> r(n);
    rc = run_plan(pl, &o, r.data());
  }
  *ms = pl->acc.msg_launches ? pl->acc.sweep_ms / (double)pl->acc.msg_launches : INFINITY;
  pl->acc = acc;
  copy_state(false);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(snap);
  if (rc) return rc;
  if (e != hipSuccess) return fail(GMOT_EDEVICE, std::string("autotune timing: ") + hipGetErrorString(e));
  return GMOT_OK;
}

constexpr double kAutotuneMargin = 0.97;

static int autotune(gmot_ctx* ctx, const std::vector<gmot_problem*>& probs, Plan** plan_io, int32_t* W_out,
                    int32_t* R_out, int32_t* H_out, double* ms_out) {
  static const NodeShape kCand[] = {{2, 1, 1}, {4, 1, 1}, {8, 1, 1},  {16, 1, 1}, {2, 2, 1}, {4, 2, 1}, {8, 2, 1},
                                    {16, 2, 1}, {4, 2, 2}, {8, 2, 2}, {16, 2, 2}, {4, 1, 2}, {8, 1, 2}, {16, 1, 2}};
  bool expl = false, any_grid = false, all_grid = true;
  for (const gmot_problem* p : probs) {
    expl = expl || p->cost_kind == GMOT_COST_EXPLICIT;
    const bool g = p->grid || p->sep_h;
    any_grid = any_grid || g;
    all_grid = all_grid && g;
  }
  std::vector<NodeShape> cands;
  // With the uniform-grid kernels on, the node shape matters only for the
  // problems they do not take; with every problem on them, one shape.  When
  // some problem admits them, every shape is also timed with them off (a small
  // plan can fill the device better through the node kernel's column ranges).
  if (all_grid) {
    cands.push_back(NodeShape{4, 1, 1, 1});
  } else {
    for (const auto& c : kCand)
      if (!expl || (c.R == 1 && c.H == 1)) cands.push_back(c);  // explicit cost: one row per lane
  }
  if (any_grid)
    for (const auto& c : kCand)
      if (!expl || (c.R == 1 && c.H == 1)) cands.push_back(NodeShape{c.W, c.R, c.H, 0});
  if (std::getenv("GMOT_NODE_SHAPE")) {  // a pinned shape is the only candidate
    NodeShape pin = choose_shape(ctx, probs);
    if (expl) pin.R = pin.H = 1;
    cands = {pin};
  }
  Plan* best = nullptr;
  double best_ms = INFINITY;
  NodeShape bWR = kDefaultShape;
  for (const auto& cand : cands) {
    Plan* pl = nullptr;
    int rc = build_plan(ctx, probs, cand, &pl);
    if (rc) {
      delete best;
      return rc;
    }
    double ms = 0;
    rc = time_plan(pl, &ms);
    if (rc) {
      delete pl;
      delete best;
      return rc;
    }
    if (std::getenv("GMOT_AUTOTUNE_LOG"))  // diagnostic: every candidate's time
      std::fprintf(stderr, "autotune W=%d R=%d H=%d grid=%d: %.4f ms per half-sweep\n", cand.W, cand.R, cand.H,
                   cand.G, ms);
    // a later candidate must be 3% faster to replace an earlier one, so
    // near-equal shapes do not flip from run to run
    if (ms < best_ms * kAutotuneMargin) {
      delete best;
      best = pl;
      best_ms = ms;
      bWR = cand;
    } else {
      delete pl;
    }
  }
  ctx->tuned[shape_key(probs)] = bWR;
  delete *plan_io;
  *plan_io = best;
  g_tiles = best->stats;
  if (W_out) *W_out = bWR.W;
  if (R_out) *R_out = bWR.R;
  if (H_out) *H_out = bWR.H;
  if (ms_out) *ms_out = best_ms;
  return GMOT_OK;
}

static int validate_opts(const gmot_opts* o) {
  if (!o) return fail(GMOT_EINVAL, "null options");
  if (!(o->tol >= 0.0)) return fail(GMOT_EINVAL, "tol must be >= 0");
  if (o->max_steps < 1) return fail(GMOT_EINVAL, "max_steps must be positive");
  if (o->check_every < 0) return fail(GMOT_EINVAL, "check_every must be >= 0");
  if (o->precision != GMOT_PREC_FP32CORE && o->precision != GMOT_PREC_FP64)
    return fail(GMOT_EINVAL, "unknown precision");
  if (o->schedule != GMOT_SCHED_LAYER && o->schedule != GMOT_SCHED_PER_NODE &&
      o->schedule != GMOT_SCHED_GAUSS_SEIDEL)
    return fail(GMOT_EINVAL, "unknown schedule");
  if (o->msg_passes != GMOT_PASSES_AUTO && o->msg_passes != GMOT_PASSES_ONE && o->msg_passes != GMOT_PASSES_TWO)
    return fail(GMOT_EINVAL, "unknown msg_passes");
  return GMOT_OK;
}

static int restart_problem(gmot_problem* p) {
  if (p->total_de > 0) HIPCHK(hipMemsetAsync(p->d_lam[0], 0, sizeof(double) * p->total_de, p->ctx->stream));
  HIPCHK(hipMemsetAsync(p->d_c, 0, sizeof(double) * kSlots * p->N, p->ctx->stream));
  p->t = 1;
  ++p->version;
  return GMOT_OK;
}

// ---------------------------------------------------------------------------
// evaluation pass (FP64)
// ---------------------------------------------------------------------------
// FP64 messages into, and node terms of, class only_class (-1: both) for every
// instance of the plan, each read from its committed slots.
static int eval_messages(Plan* pl, int only_class) {
  hipStream_t s = pl->ctx->stream;
  std::vector<int> slots(2 * pl->probs.size());
  for (size_t i = 0; i < pl->probs.size(); ++i)
    for (int c = 0; c < 2; ++c) slots[2 * i + c] = pl->probs[i]->slot_of_class(c);
  HIPCHK(hipMemcpyAsync(pl->d_inst_slot, slots.data(), sizeof(int) * slots.size(), hipMemcpyHostToDevice, s));
  // the work lists of every instance (a solve may end on thinned ones)
  if (!pl->select_lists(0)) return fail(GMOT_EDEVICE, "evaluation: full work lists missing");
  for (int c = 0; c < 2; ++c) {
    if (only_class >= 0 && c != only_class) continue;
    for (int dk = 0; dk < 4; ++dk)
      if (pl->items_general[c][dk] > 0)
        HIPCHK(launch_msg(pl->tables(c, dk), pl->items_general[c][dk], dk, pl->R, -1, s));
    // messages of the uniform-grid groups by their own kernels, in FP64
    if (!pl->tiles[c][kGridGroup].empty())
      HIPCHK(launch_msg_grid(pl->tables(c, kGridGroup), (int)pl->tiles[c][kGridGroup].size(), pl->grid_R, true, s));
    if (!pl->sep_tasks[c][0].empty()) {
      HIPCHK(launch_sep_horner(pl->tables(c, kSepHGroup), 0, (int)pl->sep_tasks[c][0].size(), true, s));
      HIPCHK(launch_sep_horner(pl->tables(c, kSepHGroup), 1, (int)pl->sep_tasks[c][1].size(), true, s));
    }
    HIPCHK(launch_node_eval(pl->tables(c, -1), (int)pl->nodes[c].size(), -1, s));
  }
  // the slot table is host memory read by a copy still in flight
  HIPCHK(hipStreamSynchronize(s));
  return GMOT_OK;
}

static EdgeDesc edge_desc(const gmot_problem* p, int e) {
  const int a = p->edges[2 * e], b = p->edges[2 * e + 1];
  EdgeDesc ed{};
  ed.supp_a = p->d_support + p->node_off[a] * p->dim;
  ed.supp_b = p->d_support + p->node_off[b] * p->dim;
  const int sa = p->slot_of_class(p->colour[a]), sb = p->slot_of_class(p->colour[b]);
  ed.lam_a = p->d_lam[sa] + p->de_off[2 * e];
  ed.lam_b = p->d_lam[sb] + p->de_off[2 * e + 1];
  ed.c_a = p->fixed[a] ? nullptr : p->d_c + kSlots * a + sa;
  ed.c_b = p->fixed[b] ? nullptr : p->d_c + kSlots * b + sb;
  ed.lg_a = p->d_lg + p->node_off[a];
  ed.lg_b = p->d_lg + p->node_off[b];
  ed.cost = p->cost_kind == GMOT_COST_EXPLICIT ? p->d_cost + p->cost_off[e] : nullptr;
  ed.n_a = p->sizes[a];
  ed.n_b = p->sizes[b];
  ed.dim = p->dim;
  ed.cost_kind = p->cost_kind;
  ed.eps = p->eps;
  return ed;
}

// FP64 objective values of the held state of every instance of a plan, in
// shared launches (outs[i] for plan instance i): the messages into both
// classes and the node terms (k_msg, k_node_eval), then the pair pass over
// every edge of every instance (k_pairs) except those of instances on the
// uniform-grid kernels, whose messages carry their plans' mean costs; the
// per-instance sums are taken on the host in the same order for any plan
// (only the column splits of the messages, and so their merge order, depend
// on the plan).
static int evaluate_plan(Plan* pl, gmot_eval* outs) {
  const size_t n = pl->probs.size();
  for (size_t i = 0; i < n; ++i) std::memset(&outs[i], 0, sizeof(gmot_eval));
  hipStream_t s = pl->ctx->stream;
  // pair pass work lists
  std::vector<EdgeDesc> eds;
  std::vector<PairItem> items;
  std::vector<int> edge0(n + 1, 0);
  for (size_t i = 0; i < n; ++i) {
    const gmot_problem* p = pl->probs[i];
    edge0[i] = (int)eds.size();
    for (int e = 0; e < p->E; ++e) {
      const int ge = (int)eds.size();
      eds.push_back(edge_desc(p, e));
      // instances on the uniform-grid kernels take their plans' sums from the
      // messages (marginals and mean costs), with no pair pass
      if (pl->inst_horner[i]) continue;
      const int na = eds.back().n_a, nb = eds.back().n_b;
      const int cw = 2048;
      for (int r0 = 0; r0 < na; r0 += kBlock)
        for (int c0 = 0; c0 < nb; c0 += cw) items.push_back({ge, r0, c0, std::min(cw, nb - c0)});
    }
  }
  edge0[n] = (int)eds.size();
  if (eds.empty()) return GMOT_OK;
  const size_t b_ed = align_up(sizeof(EdgeDesc) * eds.size(), 256);
  const size_t b_it = align_up(sizeof(PairItem) * std::max<size_t>(1, items.size()), 256);
  const size_t b_out = sizeof(double4) * std::max<size_t>(1, items.size());
  if (pl->pair_buf_size < b_ed + b_it + b_out) {
    if (pl->pair_buf) (void)hipFree(pl->pair_buf);
    pl->pair_buf = nullptr;
    pl->pair_buf_size = 0;
    if (hipMalloc(&pl->pair_buf, b_ed + b_it + b_out) != hipSuccess) return fail(GMOT_ENOMEM, "evaluation buffers");
    pl->pair_buf_size = b_ed + b_it + b_out;
  }
  char* base = (char*)pl->pair_buf;
  std::vector<double4> parts(items.size());
  std::vector<double4> ne(pl->total_nodes);
  // The pair pass reads only the committed potentials, so it runs on the
  // context's second stream (after everything issued so far on the main
  // one) beside the messages and node terms on the main stream.
  gmot_ctx* ctx = pl->ctx;
  hipError_t e1 = hipEventRecord(ctx->ev_fork, s);
  if (e1 == hipSuccess) e1 = hipStreamWaitEvent(ctx->aux, ctx->ev_fork, 0);
  if (e1 == hipSuccess)
    e1 = hipMemcpyAsync(base, eds.data(), sizeof(EdgeDesc) * eds.size(), hipMemcpyHostToDevice, ctx->aux);
  if (e1 == hipSuccess && !items.empty())
    e1 = hipMemcpyAsync(base + b_ed, items.data(), sizeof(PairItem) * items.size(), hipMemcpyHostToDevice, ctx->aux);
  if (e1 == hipSuccess)
    e1 = launch_pairs((EdgeDesc*)base, (PairItem*)(base + b_ed), (int)items.size(), (double4*)(base + b_ed + b_it),
                      ctx->aux);
  if (e1 == hipSuccess && !items.empty())
    e1 = hipMemcpyAsync(parts.data(), base + b_ed + b_it, sizeof(double4) * items.size(), hipMemcpyDeviceToHost,
                        ctx->aux);
  int rc = GMOT_OK;
  if (e1 == hipSuccess) rc = eval_messages(pl, -1);
  hipError_t e2 = hipStreamSynchronize(ctx->aux);
  if (e1 != hipSuccess) return fail(GMOT_EDEVICE, std::string("evaluation: ") + hipGetErrorString(e1));
  if (rc) return rc;
  std::vector<double4> me(pl->msgs.size());
  if (e2 == hipSuccess)
    e2 = hipMemcpyAsync(ne.data(), pl->d_node_eval, sizeof(double4) * pl->total_nodes, hipMemcpyDeviceToHost, s);
  if (e2 == hipSuccess && !me.empty())
    e2 = hipMemcpyAsync(me.data(), pl->d_msg_eval, sizeof(double4) * me.size(), hipMemcpyDeviceToHost, s);
  if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
  if (e2 != hipSuccess) return fail(GMOT_EDEVICE, std::string("evaluation: ") + hipGetErrorString(e2));
  std::vector<double> T(eds.size(), 0.0), H(eds.size(), 0.0), M(eds.size(), 0.0);
  for (size_t k = 0; k < items.size(); ++k) {
    const int e = items[k].edge;
    T[e] += parts[k].x;
    H[e] += parts[k].y;
    M[e] += parts[k].z;
  }
  // uniform-grid instances: for edge (a, b), the message into a carries the plan's
  // row sums r = q_a (mass sum r, sum r (L_(a,b) - c_a), transport sum r Cbar)
  // and the one into b its column sums; entropy sum B (log B - 1) =
  // sum r (L_(a,b) - c_a) + sum q_b (L_(b,a) - c_b) - T / eps - M
  for (size_t i = 0; i < n; ++i) {
    if (!pl->inst_horner[i]) continue;
    const gmot_problem* p = pl->probs[i];
    for (int e = 0; e < p->E; ++e) {
      const double4 ra = me[pl->de_msg[i][2 * e]], rb = me[pl->de_msg[i][2 * e + 1]];
      const int ge = edge0[i] + e;
      M[ge] = ra.x;
      T[ge] = ra.z;
      H[ge] = ra.y + rb.y - ra.z / p->eps - ra.x;
    }
  }
  for (size_t i = 0; i < n; ++i) {
    const gmot_problem* p = pl->probs[i];
    gmot_eval* out = &outs[i];
    if (p->E == 0) continue;
    double Tsum = 0, Hsum = 0, Msum = 0, mmin = INFINITY, mmax = -INFINITY;
    for (int e = edge0[i]; e < edge0[i + 1]; ++e) {
      Tsum += T[e];
      Hsum += H[e];
      Msum += M[e];
      mmin = std::min(mmin, M[e]);
      mmax = std::max(mmax, M[e]);
    }
    double err = 0, errm = 0, lin = 0, rho = 0, spread = 0, scale = p->eps * p->E;
    for (int c = 0; c < 2; ++c) {
      const int i0 = pl->inst[i].node0[c], cnt = pl->inst[i].nnodes[c];
      for (int q = i0; q < i0 + cnt; ++q) {
        const NodeItem& nd = pl->nodes[c][q];
        const double4 v = ne[nd.err_idx];
        err += v.x;
        errm = std::max(errm, v.y);
        if (nd.fixed) {
          lin += v.z;
          scale += p->eps * std::fabs(v.z);
        } else {
          rho += v.z;
          scale += p->eps * std::fabs(v.z);
          spread = std::max(spread, v.w);
        }
      }
    }
    out->dual = p->eps * (lin + rho - Msum);
    out->transport = Tsum;
    out->primal = Tsum + p->eps * Hsum;
    out->gap = out->primal - out->dual;
    out->err_sum = err;
    out->err_max = errm;
    out->mass_min = mmin;
    out->mass_max = mmax;
    out->rho_spread = spread;
    out->scale = scale;
  }
  return GMOT_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// rounding (Algorithm round)
// ---------------------------------------------------------------------------
// Device buffers of the last rounding of a problem: per directed edge the row
// sums, targets, scalings and residuals (four arrays laid out like the
// potentials), and the descriptors.  Valid while the problem's state version
// is unchanged; the rounded plans are formed from them on request.
struct RoundState {
  void* buf = nullptr;
  RoundDesc* d_desc = nullptr;          // [2E] with column weights (passes 1, 2; plan read-back)
  std::vector<int> edge_desc;           // edge -> desc index of its end in S (opposite at + E)
  std::vector<uint8_t> s_is_a;          // edge -> the end in S is the edge's first node
  std::vector<double> inv_s;            // edge -> 1 / |e_r|_1 (0 when e_r = 0)
  uint64_t version = ~0ull;
  ~RoundState() {
    if (buf) (void)hipFree(buf);
  }
};

static RoundDesc round_desc(const gmot_problem* p, int de, double* arrays) {
  const int e = de >> 1;
  const bool fwd = (de & 1) == 0;
  const int j = fwd ? p->edges[2 * e] : p->edges[2 * e + 1];
  const int k = fwd ? p->edges[2 * e + 1] : p->edges[2 * e];
  const int sj = p->slot_of_class(p->colour[j]), sk = p->slot_of_class(p->colour[k]);
  RoundDesc d{};
  d.supp_r = p->d_support + p->node_off[j] * p->dim;
  d.supp_c = p->d_support + p->node_off[k] * p->dim;
  d.lam_r = p->d_lam[sj] + p->de_off[de];
  d.lam_c = p->d_lam[sk] + p->de_off[de ^ 1];
  d.c_r = p->fixed[j] ? nullptr : p->d_c + kSlots * j + sj;
  d.c_c = p->fixed[k] ? nullptr : p->d_c + kSlots * k + sk;
  d.lg_r = p->d_lg + p->node_off[j];
  d.lg_c = p->d_lg + p->node_off[k];
  if (p->cost_kind == GMOT_COST_EXPLICIT)  // cost[y * n_j + x]: C_e^T when j = a, C_e when j = b
    d.cost = fwd ? p->d_cost + p->total_cost + p->cost_off[e] : p->d_cost + p->cost_off[e];
  const int64_t o = p->de_off[de], D = p->total_de;
  d.rs = arrays + o;
  d.tg = arrays + D + o;
  d.sc = arrays + 2 * D + o;
  d.er = arrays + 3 * D + o;
  d.n_r = p->sizes[j];
  d.n_c = p->sizes[k];
  d.dim = p->dim;
  d.cost_kind = p->cost_kind;
  d.eps = p->eps;
  return d;
}

static int round_problem(gmot_problem* p, gmot_round_result* out, double* edge_transport) {
  const int E = p->E;
  const int side = (p->t & 1) ? 0 : 1;  // the class the next half-sweep would update
  // descriptors: ends in S grouped by node (ascending neighbours), opposites at + E
  std::vector<int> sde;
  std::vector<RoundNode> nodes;
  std::vector<int> edge_desc(E, -1);
  std::vector<uint8_t> s_is_a(E, 0);
  for (int j = 0; j < p->N; ++j) {
    if (p->colour[j] != side || p->nbrs[j].empty()) continue;
    RoundNode nd{};
    nd.n = p->sizes[j];
    nd.deg = (int)p->nbrs[j].size();
    nd.d0 = (int)sde.size();
    nd.mu = p->fixed[j] ? p->d_mu + p->node_off[j] : nullptr;
    nodes.push_back(nd);
    for (int de : p->nbr_de[j]) {
      edge_desc[de >> 1] = (int)sde.size();
      s_is_a[de >> 1] = (de & 1) == 0;
      sde.push_back(de);
    }
  }
  if ((int)sde.size() != E) return fail(GMOT_ESTATE, "rounding: the tree is not bipartite as colored");
  std::vector<RoundItem> it0, it1, it2;
  for (int i = 0; i < 2 * E; ++i) {
    const int de = i < E ? sde[i] : sde[i - E] ^ 1;
    const int j = (de & 1) ? p->edges[2 * (de >> 1) + 1] : p->edges[2 * (de >> 1)];
    for (int r0 = 0; r0 < p->sizes[j]; r0 += kBlock) {
      it0.push_back({i, r0});
      (i < E ? it2 : it1).push_back({i, r0});
    }
  }
  const size_t D = (size_t)p->total_de;
  const size_t o_desc0 = align_up(sizeof(double) * 4 * D, 256);
  const size_t o_desc = o_desc0 + align_up(sizeof(RoundDesc) * 2 * E, 256);
  const size_t o_it = o_desc + align_up(sizeof(RoundDesc) * 2 * E, 256);
  const size_t n_it = it0.size() + it1.size() + it2.size();
  const size_t o_nodes = o_it + align_up(sizeof(RoundItem) * n_it, 256);
  const size_t o_part = o_nodes + align_up(sizeof(RoundNode) * nodes.size(), 256);
  const size_t o_err = o_part + align_up(sizeof(double4) * it2.size(), 256);
  const size_t total = o_err + sizeof(double) * nodes.size();
  delete p->round;
  p->round = nullptr;
  std::unique_ptr<RoundState> rs(new RoundState());
  if (hipMalloc(&rs->buf, total) != hipSuccess) return fail(GMOT_ENOMEM, "rounding buffers");
  char* base = (char*)rs->buf;
  double* arrays = (double*)base;
  std::vector<RoundDesc> d0(2 * E), d12(2 * E);
  for (int i = 0; i < 2 * E; ++i) {
    const int de = i < E ? sde[i] : sde[i - E] ^ 1;
    d0[i] = round_desc(p, de, arrays);
  }
  for (int i = 0; i < E; ++i) {
    d12[i] = d0[i];              // rows in S, pass 2: columns weighted by Y, residual e_c
    d12[i].sc_col = d0[i + E].sc;
    d12[i].er_col = d0[i + E].er;
    d12[i + E] = d0[i + E];      // rows on the other side, pass 1: columns weighted by X
    d12[i + E].sc_col = d0[i].sc;
  }
  std::vector<RoundItem> items;
  items.reserve(n_it);
  items.insert(items.end(), it0.begin(), it0.end());
  items.insert(items.end(), it1.begin(), it1.end());
  items.insert(items.end(), it2.begin(), it2.end());
  RoundDesc* dd0 = (RoundDesc*)(base + o_desc0);
  RoundDesc* dd = (RoundDesc*)(base + o_desc);
  RoundItem* di = (RoundItem*)(base + o_it);
  RoundNode* dn = (RoundNode*)(base + o_nodes);
  double4* dpart = (double4*)(base + o_part);
  double* derr = (double*)(base + o_err);
  hipStream_t s = p->ctx->stream;
  std::vector<double4> parts(it2.size());
  std::vector<double> errs(nodes.size());
  hipError_t e = hipMemcpyAsync(dd0, d0.data(), sizeof(RoundDesc) * 2 * E, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dd, d12.data(), sizeof(RoundDesc) * 2 * E, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(di, items.data(), sizeof(RoundItem) * n_it, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dn, nodes.data(), sizeof(RoundNode) * nodes.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_round_rows(0, dd0, di, (int)it0.size(), nullptr, s);
  if (e == hipSuccess) e = launch_round_node(dn, (int)nodes.size(), dd0, derr, s);
  if (e == hipSuccess) e = launch_round_rows(1, dd, di + it0.size(), (int)it1.size(), nullptr, s);
  if (e == hipSuccess) e = launch_round_rows(2, dd, di + it0.size() + it1.size(), (int)it2.size(), dpart, s);
  if (e == hipSuccess) e = hipMemcpyAsync(parts.data(), dpart, sizeof(double4) * parts.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(errs.data(), derr, sizeof(double) * errs.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(GMOT_EDEVICE, std::string("rounding: ") + hipGetErrorString(e));
  // per edge: transport of F, bilinear term, |e_r|_1, in the order of the items
  std::vector<double> T(E, 0.0), Bl(E, 0.0), Se(E, 0.0);
  double cinf = 0.0;
  for (size_t i = 0; i < it2.size(); ++i) {
    const int edge = sde[it2[i].desc] >> 1;
    T[edge] += parts[i].x;
    Bl[edge] += parts[i].y;
    Se[edge] += parts[i].z;
    cinf = std::max(cinf, parts[i].w);
  }
  rs->inv_s.assign(E, 0.0);
  double tot = 0.0;
  for (int edge = 0; edge < E; ++edge) {
    if (Se[edge] > 0.0) rs->inv_s[edge] = 1.0 / Se[edge];
    const double te = T[edge] + Bl[edge] * rs->inv_s[edge];
    if (edge_transport) edge_transport[edge] = te;
    tot += te;
  }
  double err = 0.0;
  for (double v : errs) err += v;
  out->transport = tot;
  out->err_side = err;
  out->c_inf = cinf;
  out->side = side;
  out->reserved = 0;
  rs->d_desc = dd;
  rs->edge_desc = std::move(edge_desc);
  rs->s_is_a = std::move(s_is_a);
  rs->version = p->version;
  p->round = rs.release();
  return GMOT_OK;
}

void gmot_ctx_retain(gmot_ctx* ctx) { ctx->refs.fetch_add(1, std::memory_order_relaxed); }

void gmot_ctx_release(gmot_ctx* ctx) {
  if (!ctx || ctx->refs.fetch_sub(1, std::memory_order_acq_rel) != 1) return;
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

// Stopping sum over every node (both classes) of the plan's first instance,
// FP64 from the committed slots (eval_messages), summed as evaluate_plan sums it.
static int stopping_sum(Plan* pl, double* e_sum, double* e_max) {
  int rc = eval_messages(pl, -1);
  if (rc) return rc;
  std::vector<double4> ne(std::max(1, pl->total_nodes));
  HIPCHK(hipMemcpy(ne.data(), pl->d_node_eval, sizeof(double4) * pl->total_nodes, hipMemcpyDeviceToHost));
  double err = 0.0, errm = 0.0;
  for (int c = 0; c < 2; ++c) {
    const int i0 = pl->inst[0].node0[c], cnt = pl->inst[0].nnodes[c];
    for (int q = i0; q < i0 + cnt; ++q) {
      const double4 v = ne[pl->nodes[c][q].err_idx];
      err += v.x;
      errm = std::max(errm, v.y);
    }
  }
  *e_sum = err;
  *e_max = errm;
  return GMOT_OK;
}

// Node-sequential (Gauss-Seidel) sweeps: every node with neighbours, in
// breadth-first order from node 0, takes the per-node update of Algorithm
// tree_local_reg from its neighbours' committed potentials -- the FP64
// message kernel over that node's messages alone (k_msg, its plan items),
// then k_gs_update -- written in place into its class's committed slot, so
// the nodes after it in the sweep read it.  The stop test is the FP64
// stopping sum over every node, before the first sweep and after every
// check_every sweeps (4 by default); steps counts sweeps, t is unchanged.
static int solve_gauss_seidel(gmot_problem* p, const gmot_opts* o, gmot_result* out) {
  Plan* pl = p->plan;
  std::memset(out, 0, sizeof(*out));
  out->t = p->t;
  if (p->E == 0) {
    out->status = GMOT_CONVERGED;
    return GMOT_OK;
  }
  hipStream_t s = p->ctx->stream;
  struct Step { int c, item, dk, first, count; };
  std::vector<Step> steps;
  std::map<int, int> item_of[2];
  for (int c = 0; c < 2; ++c)
    for (size_t i = 0; i < pl->nodes[c].size(); ++i) item_of[c][pl->nodes[c][i].node] = (int)i;
  std::vector<char> seen(p->N, 0);
  std::deque<int> dq{0};
  seen[0] = 1;
  while (!dq.empty()) {
    const int v = dq.front();
    dq.pop_front();
    if (!p->nbrs[v].empty()) {
      const int c = p->colour[v], item = item_of[c].at(v);
      const NodeItem& nd = pl->nodes[c][item];
      const int dk = p->cost_kind == GMOT_COST_EXPLICIT ? 0 : p->dim;
      int count = 0;
      for (int m = nd.msg0; m < nd.msg0 + nd.deg; ++m) count += pl->msg_item_range[m].second;
      steps.push_back({c, item, dk, pl->msg_item_range[nd.msg0].first, count});
    }
    for (int w : p->nbrs[v])
      if (!seen[w]) {
        seen[w] = 1;
        dq.push_back(w);
      }
  }
  const int every = o->check_every > 0 ? o->check_every : 4;
  // messages into class c read the other class's committed slot; updates go
  // to class c's committed slot
  const int src_slot[2] = {p->slot_of_class(1), p->slot_of_class(0)};
  const int dst_slot[2] = {p->slot_of_class(0), p->slot_of_class(1)};
  const auto t0 = std::chrono::steady_clock::now();
  int64_t sweeps = 0;
  double E = INFINITY, Em = 0.0;
  int status = GMOT_NOT_CONVERGED;
  for (;;) {
    if (sweeps % every == 0 || sweeps >= o->max_steps) {
      int rc = stopping_sum(pl, &E, &Em);
      if (rc) return rc;
      if (!std::isfinite(E)) {
        status = GMOT_NONFINITE;
        break;
      }
      if (E <= o->tol) {
        status = GMOT_CONVERGED;
        break;
      }
      if (sweeps >= o->max_steps) break;
    }
    for (const Step& g : steps) {
      Tables tb = pl->tables(g.c, g.dk);
      tb.items += g.first;
      HIPCHK(launch_msg(tb, g.count, g.dk, pl->R, src_slot[g.c], s));
      HIPCHK(launch_gs_update(pl->tables(g.c, -1), g.item, dst_slot[g.c], s));
    }
    ++sweeps;
    ++p->version;
  }
  out->status = status;
  out->steps = sweeps;
  out->t = p->t;
  out->err_sum = E;
  out->err_max = Em;
  out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return GMOT_OK;
}

extern "C" {

int gmot_ctx_create(gmot_ctx** out, int device, void* hip_stream) {
  if (!out) return fail(GMOT_EINVAL, "null output");
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return fail(GMOT_EDEVICE, "no HIP device");
  if (device < 0 || device >= count) return fail(GMOT_EINVAL, "device index out of range");
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(GMOT_EDEVICE, std::string("libgmot is built for gfx950, found ") + prop.gcnArchName);
  HIPCHK(hipSetDevice(device));
  std::unique_ptr<gmot_ctx> c(new gmot_ctx());
  c->device = device;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
    c->clk_hz = 1000.0 * khz;
  HIPCHK(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  *out = c.release();
  return GMOT_OK;
}

void gmot_ctx_destroy(gmot_ctx* ctx) { gmot_ctx_release(ctx); }


int gmot_problem_create(gmot_ctx* ctx, const gmot_tree_desc* desc, int32_t first_color, gmot_problem** out) {
  if (!ctx || !out) return fail(GMOT_EINVAL, "null context or output");
  std::unique_ptr<gmot_problem> p(new gmot_problem());
  p->ctx = ctx;
  int rc = validate_and_copy(desc, p.get(), first_color);
  if (rc) return rc;
  HIPCHK(hipSetDevice(ctx->device));
  rc = upload(desc, p.get());
  if (rc) {
    if (p->arena) (void)hipFree(p->arena);
    if (p->d_cost_tile) (void)hipFree(p->d_cost_tile);
    return rc;
  }
  gmot_ctx_retain(ctx);
  *out = p.release();
  return GMOT_OK;
}

int gmot_junction_create(gmot_ctx* ctx, const gmot_junction_desc* d, int32_t first_color, gmot_problem** out) {
  if (!ctx || !d || !out) return fail(GMOT_EINVAL, "null argument");
  if (d->n_vars < 1 || d->n_seps < 1 || !d->var_sizes || !d->sep_nvars || !d->sep_vars || !d->sep_fixed)
    return fail(GMOT_EINVAL, "a junction tree needs variables and separators");
  if (d->n_cliques != d->n_seps - 1) return fail(GMOT_EINVAL, "a junction tree has one clique fewer than separators");
  if (d->n_cliques > 0 && (!d->cliques || !d->clique_cost)) return fail(GMOT_EINVAL, "null clique arrays");
  for (int v = 0; v < d->n_vars; ++v)
    if (d->var_sizes[v] < 1) return fail(GMOT_EINVAL, "a variable needs at least one support point");
  // every variable in exactly one separator; joint state counts per separator
  std::vector<int> owner(d->n_vars, -1);
  std::vector<int32_t> sizes(d->n_seps, 1);
  int64_t o = 0;
  for (int s = 0; s < d->n_seps; ++s) {
    if (d->sep_nvars[s] < 1) return fail(GMOT_EINVAL, "a separator needs at least one variable");
    int64_t states = 1;
    for (int i = 0; i < d->sep_nvars[s]; ++i) {
      const int v = d->sep_vars[o + i];
      if (v < 0 || v >= d->n_vars) return fail(GMOT_EINVAL, "separator variable index out of range");
      if (owner[v] >= 0) return fail(GMOT_EINVAL, "a variable may belong to one separator only");
      owner[v] = s;
      states *= d->var_sizes[v];
      if (states > INT32_MAX) return fail(GMOT_EINVAL, "too many joint states in a separator");
    }
    o += d->sep_nvars[s];
    sizes[s] = (int32_t)states;
  }
  for (int v = 0; v < d->n_vars; ++v)
    if (owner[v] < 0) return fail(GMOT_EINVAL, "every variable must belong to a separator");
  // the tree over separators: edges are the cliques, costs their tensors read as matrices
  gmot_tree_desc td{};
  td.n_nodes = d->n_seps;
  td.n_edges = d->n_cliques;
  td.edges = d->cliques;
  td.sizes = sizes.data();
  td.dim = 1;
  td.support = nullptr;
  td.is_fixed = d->sep_fixed;
  td.marginal = d->sep_marginal;
  td.cost_kind = GMOT_COST_EXPLICIT;
  td.cost = d->clique_cost;
  td.eps = d->eps;
  return gmot_problem_create(ctx, &td, first_color, out);
}

void gmot_problem_destroy(gmot_problem* p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->ctx->stream);
  delete p->plan;
  delete p->round;
  if (p->arena) (void)hipFree(p->arena);
  if (p->d_cost_tile) (void)hipFree(p->d_cost_tile);
  gmot_ctx* ctx = p->ctx;
  delete p;
  gmot_ctx_release(ctx);
}

int gmot_solve(gmot_problem* p, const gmot_opts* o, gmot_result* out) {
  if (!p || !out) return fail(GMOT_EINVAL, "null problem or result");
  int rc = validate_opts(o);
  if (rc) return rc;
  HIPCHK(hipSetDevice(p->ctx->device));
  if (o->restart) {
    rc = restart_problem(p);
    if (rc) return rc;
  }
  rc = ensure_plan(p);
  if (rc) return rc;
  if (o->schedule == GMOT_SCHED_GAUSS_SEIDEL) return solve_gauss_seidel(p, o, out);
  return solve_plan(p->plan, o, out);
}

int gmot_evaluate(gmot_problem* p, gmot_eval* out) {
  if (!p || !out) return fail(GMOT_EINVAL, "null problem or output");
  std::memset(out, 0, sizeof(*out));
  if (p->E == 0) return GMOT_OK;
  HIPCHK(hipSetDevice(p->ctx->device));
  int rc = ensure_plan(p);
  if (rc) return rc;
  return evaluate_plan(p->plan, out);
}

int gmot_round(gmot_problem* p, gmot_round_result* out, double* edge_transport) {
  if (!p || !out) return fail(GMOT_EINVAL, "null problem or output");
  std::memset(out, 0, sizeof(*out));
  out->side = (p->t & 1) ? 0 : 1;
  if (p->E == 0) return GMOT_OK;
  if (p->t < 2) return fail(GMOT_ESTATE, "rounding needs a state produced by at least one half-sweep");
  HIPCHK(hipSetDevice(p->ctx->device));
  return round_problem(p, out, edge_transport);
}

int gmot_get_rounded_coupling(gmot_problem* p, int32_t edge, double* out) {
  if (!p || !out) return fail(GMOT_EINVAL, "null problem or output");
  if (edge < 0 || edge >= p->E) return fail(GMOT_EINVAL, "edge index out of range");
  if (!p->round || p->round->version != p->version)
    return fail(GMOT_ESTATE, "no rounding of the held state: call gmot_round first");
  HIPCHK(hipSetDevice(p->ctx->device));
  const RoundState* rs = p->round;
  const int i = rs->edge_desc[edge];
  const size_t total = (size_t)p->sizes[p->edges[2 * edge]] * p->sizes[p->edges[2 * edge + 1]];
  double* buf = nullptr;
  if (hipMalloc(&buf, sizeof(double) * std::max<size_t>(1, total)) != hipSuccess)
    return fail(GMOT_ENOMEM, "rounded plan buffer");
  hipStream_t s = p->ctx->stream;
  hipError_t e = launch_round_plan(rs->d_desc + i, rs->d_desc + i + p->E, rs->inv_s[edge], rs->s_is_a[edge], buf,
                                   total, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out, buf, sizeof(double) * total, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (e != hipSuccess) return fail(GMOT_EDEVICE, std::string("rounded plan: ") + hipGetErrorString(e));
  return GMOT_OK;
}

int64_t gmot_potentials_size(const gmot_problem* p) { return p ? p->total_de : -1; }

int gmot_get_potentials(gmot_problem* p, double* out) {
  if (!p || (!out && p->total_de > 0)) return fail(GMOT_EINVAL, "null problem or output");
  if (p->total_de == 0) return GMOT_OK;
  HIPCHK(hipSetDevice(p->ctx->device));
  // Lam_(j,k) = L_(j,k) - c_j with both read from node j's committed slot
  std::vector<double> sv[kSlots], cv(kSlots * p->N);
  HIPCHK(hipStreamSynchronize(p->ctx->stream));
  for (int q = 0; q < kSlots; ++q) {
    sv[q].resize(p->total_de);
    HIPCHK(hipMemcpy(sv[q].data(), p->d_lam[q], sizeof(double) * p->total_de, hipMemcpyDeviceToHost));
  }
  HIPCHK(hipMemcpy(cv.data(), p->d_c, sizeof(double) * kSlots * p->N, hipMemcpyDeviceToHost));
  for (int de = 0; de < 2 * p->E; ++de) {
    const int e = de >> 1;
    const int j = (de & 1) ? p->edges[2 * e + 1] : p->edges[2 * e];
    const int slot = p->slot_of_class(p->colour[j]);
    const std::vector<double>& src = sv[slot];
    const double c = p->fixed[j] ? 0.0 : cv[kSlots * j + slot];
    for (int64_t i = p->de_off[de]; i < p->de_off[de + 1]; ++i) out[i] = src[i] - c;
  }
  return GMOT_OK;
}

int gmot_get_potentials_dev(gmot_problem* p, double* out_dev) {
  if (!p || (!out_dev && p->total_de > 0)) return fail(GMOT_EINVAL, "null problem or output");
  if (p->total_de == 0) return GMOT_OK;
  HIPCHK(hipSetDevice(p->ctx->device));
  std::vector<SegCopy> segs(2 * p->E);
  for (int de = 0; de < 2 * p->E; ++de) {
    const int e = de >> 1;
    const int j = (de & 1) ? p->edges[2 * e + 1] : p->edges[2 * e];
    const int slot = p->slot_of_class(p->colour[j]);
    segs[de] = {p->d_lam[slot] + p->de_off[de], out_dev + p->de_off[de],
                p->fixed[j] ? nullptr : p->d_c + kSlots * j + slot, p->de_off[de + 1] - p->de_off[de]};
  }
  void* buf = nullptr;
  if (hipMalloc(&buf, sizeof(SegCopy) * segs.size()) != hipSuccess) return fail(GMOT_ENOMEM, "copy table");
  hipError_t e = hipMemcpyAsync(buf, segs.data(), sizeof(SegCopy) * segs.size(), hipMemcpyHostToDevice,
                                p->ctx->stream);
  if (e == hipSuccess) e = launch_seg_copy((const SegCopy*)buf, (int)segs.size(), p->ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->ctx->stream);
  (void)hipFree(buf);
  if (e != hipSuccess) return fail(GMOT_EDEVICE, std::string("potential read-back: ") + hipGetErrorString(e));
  return GMOT_OK;
}

int gmot_set_potentials(gmot_problem* p, const double* in) {
  if (!p || (!in && p->total_de > 0)) return fail(GMOT_EINVAL, "null problem or input");
  for (int64_t i = 0; i < p->total_de; ++i)
    if (!std::isfinite(in[i])) return fail(GMOT_EINVAL, "non-finite potential");
  HIPCHK(hipSetDevice(p->ctx->device));
  HIPCHK(hipStreamSynchronize(p->ctx->stream));
  if (p->total_de) HIPCHK(hipMemcpy(p->d_lam[0], in, sizeof(double) * p->total_de, hipMemcpyHostToDevice));
  HIPCHK(hipMemset(p->d_c, 0, sizeof(double) * kSlots * p->N));
  HIPCHK(hipDeviceSynchronize());
  p->t = 1;
  ++p->version;
  return GMOT_OK;
}

int gmot_set_potentials_dev(gmot_problem* p, const double* in_dev) {
  if (!p || (!in_dev && p->total_de > 0)) return fail(GMOT_EINVAL, "null problem or input");
  HIPCHK(hipSetDevice(p->ctx->device));
  if (p->total_de)
    HIPCHK(hipMemcpyAsync(p->d_lam[0], in_dev, sizeof(double) * p->total_de, hipMemcpyDeviceToDevice,
                          p->ctx->stream));
  HIPCHK(hipMemsetAsync(p->d_c, 0, sizeof(double) * kSlots * p->N, p->ctx->stream));
  p->t = 1;
  ++p->version;
  return GMOT_OK;
}

int gmot_get_coupling(gmot_problem* p, int32_t edge, double* out) {
  if (!p || !out) return fail(GMOT_EINVAL, "null problem or output");
  if (edge < 0 || edge >= p->E) return fail(GMOT_EINVAL, "edge index out of range");
  HIPCHK(hipSetDevice(p->ctx->device));
  const EdgeDesc ed = edge_desc(p, edge);
  const size_t total = (size_t)ed.n_a * ed.n_b;
  void* buf = nullptr;
  if (hipMalloc(&buf, 256 + sizeof(double) * total) != hipSuccess) return fail(GMOT_ENOMEM, "coupling buffer");
  hipStream_t s = p->ctx->stream;
  hipError_t e = hipMemcpyAsync(buf, &ed, sizeof(ed), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_coupling((EdgeDesc*)buf, (double*)((char*)buf + 256), total, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out, (char*)buf + 256, sizeof(double) * total, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (e != hipSuccess) return fail(GMOT_EDEVICE, std::string("coupling: ") + hipGetErrorString(e));
  return GMOT_OK;
}

int gmot_get_node_marginal(gmot_problem* p, int32_t node, double* out) {
  if (!p || !out) return fail(GMOT_EINVAL, "null problem or output");
  if (node < 0 || node >= p->N) return fail(GMOT_EINVAL, "node index out of range");
  if (p->E == 0) {
    if (!p->fixed[node]) return fail(GMOT_EINVAL, "a lone free node has no marginal");
    HIPCHK(hipMemcpy(out, p->d_mu, sizeof(double) * p->sizes[0], hipMemcpyDeviceToHost));
    return GMOT_OK;
  }
  HIPCHK(hipSetDevice(p->ctx->device));
  int rc = ensure_plan(p);
  if (rc) return rc;
  rc = eval_messages(p->plan, p->colour[node]);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(p->ctx->stream));
  HIPCHK(hipMemcpy(out, p->d_qbar + p->node_off[node], sizeof(double) * p->sizes[node], hipMemcpyDeviceToHost));
  return GMOT_OK;
}

struct gmot_batch {
  gmot_ctx* ctx = nullptr;
  std::vector<gmot_problem*> probs;
  Plan* plan = nullptr;
  // the cold restart's segments (every instance's first potential slot and
  // normalisers), uploaded on the first restart
  ZeroSeg* d_zero = nullptr;
  int n_zero = 0;
};

int gmot_batch_create(gmot_ctx* ctx, gmot_problem* const* probs, int32_t count, gmot_batch** out) {
  if (!ctx || !probs || !out || count < 1) return fail(GMOT_EINVAL, "bad batch arguments");
  std::unique_ptr<gmot_batch> b(new gmot_batch());
  b->ctx = ctx;
  for (int i = 0; i < count; ++i) {
    if (!probs[i]) return fail(GMOT_EINVAL, "null problem in batch");
    if (probs[i]->ctx != ctx) return fail(GMOT_ESTATE, "batch mixes contexts");
    b->probs.push_back(probs[i]);
  }
  HIPCHK(hipSetDevice(ctx->device));
  int rc = build_plan(ctx, b->probs, choose_shape(ctx, b->probs), &b->plan);
  if (rc) return rc;
  gmot_ctx_retain(ctx);
  *out = b.release();
  return GMOT_OK;
}

void gmot_batch_destroy(gmot_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->ctx->stream);
  delete b->plan;
  if (b->d_zero) (void)hipFree(b->d_zero);
  gmot_ctx* ctx = b->ctx;
  delete b;
  gmot_ctx_release(ctx);
}

int gmot_batch_solve(gmot_batch* b, const gmot_opts* o, gmot_result* outs) {
  if (!b || !outs) return fail(GMOT_EINVAL, "null batch or results");
  int rc = validate_opts(o);
  if (rc) return rc;
  if (o->schedule == GMOT_SCHED_GAUSS_SEIDEL)
    return fail(GMOT_ENOTSUP, "the Gauss-Seidel schedule runs one problem at a time (gmot_solve)");
  HIPCHK(hipSetDevice(b->ctx->device));
  if (o->restart) {
    // what restart_problem clears, for every instance in one launch
    if (!b->d_zero) {
      std::vector<ZeroSeg> segs;
      for (gmot_problem* p : b->probs) {
        if (p->total_de > 0) segs.push_back({p->d_lam[0], (int64_t)p->total_de});
        segs.push_back({p->d_c, (int64_t)kSlots * p->N});
      }
      if (hipMalloc(&b->d_zero, sizeof(ZeroSeg) * segs.size()) != hipSuccess) {
        b->d_zero = nullptr;
        return fail(GMOT_ENOMEM, "restart segments");
      }
      HIPCHK(hipMemcpy(b->d_zero, segs.data(), sizeof(ZeroSeg) * segs.size(), hipMemcpyHostToDevice));
      b->n_zero = (int)segs.size();
    }
    HIPCHK(launch_zero_segs(b->d_zero, b->n_zero, b->ctx->stream));
    for (gmot_problem* p : b->probs) {
      p->t = 1;
      ++p->version;
    }
  }
  return solve_plan(b->plan, o, outs);
}

int gmot_batch_evaluate(gmot_batch* b, gmot_eval* outs) {
  if (!b || !outs) return fail(GMOT_EINVAL, "null batch or output");
  HIPCHK(hipSetDevice(b->ctx->device));
  return evaluate_plan(b->plan, outs);
}

int gmot_problem_autotune(gmot_problem* p, int32_t* waves_per_block, int32_t* rows_per_lane, int32_t* lane_groups,
                          double* best_ms) {
  if (!p) return fail(GMOT_EINVAL, "null problem");
  if (p->E == 0) return GMOT_OK;
  HIPCHK(hipSetDevice(p->ctx->device));
  return autotune(p->ctx, {p}, &p->plan, waves_per_block, rows_per_lane, lane_groups, best_ms);
}

int gmot_batch_autotune(gmot_batch* b, int32_t* waves_per_block, int32_t* rows_per_lane, int32_t* lane_groups,
                        double* best_ms) {
  if (!b) return fail(GMOT_EINVAL, "null batch");
  HIPCHK(hipSetDevice(b->ctx->device));
  return autotune(b->ctx, b->probs, &b->plan, waves_per_block, rows_per_lane, lane_groups, best_ms);
}

// ---- star warm-start data movement ------------------------------------------
static int star_descs(gmot_problem* const* probs, int32_t count, int* L_out, int* n_out, StarDesc** d_out,
                      int** d_rejected, ZeroSeg** d_zero = nullptr) {
  if (!probs || count < 1) return fail(GMOT_EINVAL, "no problems");
  gmot_ctx* ctx = probs[0]->ctx;
  int L = -1, n = -1;
  std::vector<StarDesc> h(count);
  std::vector<ZeroSeg> zs(count);  // every instance's normalisers (cleared by the warm start)
  for (int i = 0; i < count; ++i) {
    const gmot_problem* p = probs[i];
    if (!p || p->ctx != ctx) return fail(GMOT_ESTATE, "problems must share one context");
    bool ok = p->E >= 1 && p->N == p->E + 1 && !p->fixed[0] && p->first_color == 0 &&
              p->cost_kind == GMOT_COST_SQEUCLID;
    for (int e = 0; ok && e < p->E; ++e) ok = p->edges[2 * e] == 0 && p->edges[2 * e + 1] == e + 1;
    for (int j = 1; ok && j < p->N; ++j) ok = p->fixed[j] && p->sizes[j] == p->sizes[0];
    if (!ok) return fail(GMOT_EINVAL, "warm start needs star instances (free center 0, edges (0,l), equal sizes)");
    if (L < 0) {
      L = p->E;
      n = p->sizes[0];
    }
    if (p->E != L || p->sizes[0] != n) return fail(GMOT_EINVAL, "star instances of one call must share L and n");
    h[i].lg_leaf = p->d_lg + p->node_off[1];
    h[i].lam0 = p->d_lam[0] + p->de_off[0];
    h[i].lam_cur = p->d_lam[p->slot_of_class(p->colour[1])] + p->de_off[0];
    zs[i] = {p->d_c, (int64_t)kSlots * p->N};
  }
  // scratch: the star table, the rejection counter, the segment table
  const size_t o_zero = align_up(sizeof(StarDesc) * count, 256) + 256;
  const size_t need = o_zero + sizeof(ZeroSeg) * count;
  if (ctx->scratch_size < need) {
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    ctx->scratch = nullptr;
    ctx->scratch_size = 0;
    if (hipMalloc(&ctx->scratch, need) != hipSuccess) return fail(GMOT_ENOMEM, "warm-start tables");
    ctx->scratch_size = need;
  }
  StarDesc* d = (StarDesc*)ctx->scratch;
  // earlier launches may still read the scratch tables: wait, then copy synchronously
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipMemcpy(d, h.data(), sizeof(StarDesc) * count, hipMemcpyHostToDevice));
  if (d_zero) {
    *d_zero = (ZeroSeg*)((char*)ctx->scratch + o_zero);
    HIPCHK(hipMemcpy(*d_zero, zs.data(), sizeof(ZeroSeg) * count, hipMemcpyHostToDevice));
  }
  *L_out = L;
  *n_out = n;
  *d_out = d;
  if (d_rejected) *d_rejected = (int*)((char*)ctx->scratch + align_up(sizeof(StarDesc) * count, 256));
  return GMOT_OK;
}

int gmot_star_features_dev(gmot_problem* const* probs, int32_t count, float shift, float scale, float* x_dev) {
  if (!x_dev) return fail(GMOT_EINVAL, "null output");
  int L, n;
  StarDesc* d;
  int rc = star_descs(probs, count, &L, &n, &d, nullptr);
  if (rc) return rc;
  HIPCHK(launch_star_features(d, count, L, n, shift, scale, x_dev, probs[0]->ctx->stream));
  return GMOT_OK;
}

int gmot_star_targets_dev(gmot_problem* const* probs, int32_t count, float out_scale, float* t_dev) {
  if (!t_dev || !(out_scale > 0.f)) return fail(GMOT_EINVAL, "null output or non-positive scale");
  int L, n;
  StarDesc* d;
  int rc = star_descs(probs, count, &L, &n, &d, nullptr);
  if (rc) return rc;
  HIPCHK(launch_star_targets(d, count, L, n, out_scale, t_dev, probs[0]->ctx->stream));
  return GMOT_OK;
}

int gmot_star_apply_dev(gmot_problem* const* probs, int32_t count, const float* y_dev, float out_scale,
                        int32_t* rejected) {
  if (!y_dev) return fail(GMOT_EINVAL, "null prediction");
  int L, n;
  StarDesc* d;
  int* d_rej = nullptr;
  ZeroSeg* d_zero = nullptr;
  int rc = star_descs(probs, count, &L, &n, &d, &d_rej, &d_zero);
  if (rc) return rc;
  hipStream_t s = probs[0]->ctx->stream;
  HIPCHK(hipMemsetAsync(d_rej, 0, sizeof(int), s));
  HIPCHK(launch_zero_segs(d_zero, count, s));
  HIPCHK(launch_star_apply(d, count, L, n, y_dev, out_scale, d_rej, s));
  int rej = 0;
  HIPCHK(hipMemcpyAsync(&rej, d_rej, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int i = 0; i < count; ++i) {
    probs[i]->t = 1;
    ++probs[i]->version;
  }
  if (rejected) *rejected = rej;
  return GMOT_OK;
}

int gmot_mlp_warm_start(gmot_mlp* m, gmot_problem* const* probs, int32_t count, float shift, float scale,
                        float out_scale, int32_t* rejected) {
  if (!m || !probs || count < 1) return fail(GMOT_EINVAL, "null network or problems");
  int n_in = 0, n_out = 0;
  gmot_mlp_widths(m, &n_in, &n_out);
  const int B = (count + 7) / 8 * 8;
  float *x = nullptr, *y = nullptr;
  int rc = gmot_mlp_workspace(m, B, &x, &y);
  if (rc) return fail(rc, gmot_mlp_last_error());
  int L, n;
  StarDesc* d;
  rc = star_descs(probs, count, &L, &n, &d, nullptr);
  if (rc) return rc;
  if (L * n != n_in || L * n != n_out) return fail(GMOT_EINVAL, "network widths do not match L * n");
  hipStream_t s = probs[0]->ctx->stream;
  if (B > count) HIPCHK(hipMemsetAsync(x + (size_t)count * n_in, 0, sizeof(float) * (size_t)(B - count) * n_in, s));
  HIPCHK(launch_star_features(d, count, L, n, shift, scale, x, s));
  rc = gmot_mlp_forward_dev(m, x, B, y);
  if (rc) return fail(rc, gmot_mlp_last_error());
  return gmot_star_apply_dev(probs, count, y, out_scale, rejected);
}

static int copy_stats(Plan* pl, gmot_stats* out, int32_t reset) {
  if (!out) return fail(GMOT_EINVAL, "null output");
  if (!pl) {
    std::memset(out, 0, sizeof(*out));
    return GMOT_OK;
  }
  *out = pl->acc;
  if (reset) pl->acc = gmot_stats{};
  return GMOT_OK;
}

int gmot_problem_stats(gmot_problem* p, gmot_stats* out, int32_t reset) {
  if (!p) return fail(GMOT_EINVAL, "null problem");
  return copy_stats(p->plan, out, reset);
}

int gmot_batch_stats(gmot_batch* b, gmot_stats* out, int32_t reset) {
  if (!b) return fail(GMOT_EINVAL, "null batch");
  return copy_stats(b->plan, out, reset);
}

const char* gmot_strerror(int code) {
  switch (code) {
    case GMOT_OK: return "ok";
    case GMOT_EINVAL: return "invalid argument";
    case GMOT_EMARGINAL: return "invalid marginal";
    case GMOT_ENOMEM: return "out of memory";
    case GMOT_EDEVICE: return "device error";
    case GMOT_ENOTSUP: return "not supported";
    case GMOT_ESTATE: return "invalid state";
    default: return "unknown error";
  }
}

const char* gmot_last_error(void) { return g_last_error.c_str(); }

int gmot_last_tiles(int32_t* rows_per_block, int32_t* waves_per_block, int32_t* blocks_c0, int32_t* blocks_c1) {
  if (rows_per_block) *rows_per_block = g_tiles.rows;
  if (waves_per_block) *waves_per_block = g_tiles.max_splits;
  if (blocks_c0) *blocks_c0 = g_tiles.blocks[0];
  if (blocks_c1) *blocks_c1 = g_tiles.blocks[1];
  return GMOT_OK;
}

}  // extern "C"
