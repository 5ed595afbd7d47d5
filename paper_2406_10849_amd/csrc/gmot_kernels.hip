// gfx950 kernels of the bipartite iterative-scaling hot path.
//
//   k_node     -- one half-sweep's work for a 64-row tile of a node of the
//                 class being updated: the message log-sum-exps of every
//                 incident edge (the K u products of Theorem tree_dual_var,
//                 eq. q), the stopping-sum terms of the state before the update
//                 (Algorithm tree_local_reg; Lemma f_upper_bound_tree for the
//                 arithmetic mean) and the update of eq. bipartite_tree_updates1/2
//                 in its closed form (Prop. equi).
//   k_finalize -- per instance: node normalisers, stopping sum, stop decision.
//   k_msg             -- FP64 message LSE with given slots (evaluation).
//   k_node_eval       -- evaluation: merge, stopping-sum terms, <Lam, mu> / rho.
//   k_pairs           -- FP64 transport / entropy / mass sums of every plan
//                        (eq. bi-marginal_B_sol, eq. ot_graph_pairwise_mass).
//   k_coupling        -- one plan written out in FP64.
//
// Arithmetic contract of the FP32-core node kernel: FP64 potentials, FP64
// exponent arguments (w - row max), FP32 v_exp_f32 on the reduced argument,
// pairs of FP32 terms added in FP32 and accumulated in FP64, FP64 merge, log,
// stopping-sum terms and node normalisers.
#include "gmot_internal.h"

#include <cmath>
#include <type_traits>

namespace gmot {

namespace {


// Wave reductions without the LDS crossbar: within each row of 16 lanes, DPP
// moves pair lane i with i ^ 1, i ^ 2 (quad permutes), 7 - i within each half
// row and 15 - i within the row, so every lane ends with its row's total (the
// same bits in all 16 lanes: each step adds two equal-order partials); the four
// row totals are then read with v_readlane and combined in a fixed order.
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)(b & 0xffffffff), (int)(b & 0xffffffff), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double lane_read(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;
__device__ inline double wave_sum(double v) {
  v += dpp_move<kDppXor1>(v);
  v += dpp_move<kDppXor2>(v);
  v += dpp_move<kDppHalfMirror>(v);
  v += dpp_move<kDppMirror>(v);
  return ((lane_read(v, 0) + lane_read(v, 16)) + lane_read(v, 32)) + lane_read(v, 48);
}
__device__ inline double wave_max(double v) {
  v = fmax(v, dpp_move<kDppXor1>(v));
  v = fmax(v, dpp_move<kDppXor2>(v));
  v = fmax(v, dpp_move<kDppHalfMirror>(v));
  v = fmax(v, dpp_move<kDppMirror>(v));
  return fmax(fmax(lane_read(v, 0), lane_read(v, 16)), fmax(lane_read(v, 32), lane_read(v, 48)));
}

// A free node's normaliser c_j = LSE over its tile records of the (max,
// scaled sum) pairs of abar at record entry col: tiles lane, lane + 64, ...
// per lane, then a wave max and a wave sum, so every caller gets the same
// bits.  (m0, s0) are the pair of tile `lane`, loaded by the caller (any
// value when lane >= tiles); every lane returns c_j.
__device__ inline double tile_lse(const double* __restrict__ tp, int tiles, int stride, int col, double m0,
                                  double s0) {
  const int lane = threadIdx.x & 63;
  if (lane >= tiles) m0 = -INFINITY;
  double M = m0;
  for (int tt = lane + 64; tt < tiles; tt += 64) M = fmax(M, tp[(size_t)tt * stride + col]);
  M = wave_max(M);
  double S = (m0 > -INFINITY) ? s0 * exp(m0 - M) : 0.0;
  for (int tt = lane + 64; tt < tiles; tt += 64) {
    const double mt = tp[(size_t)tt * stride + col];
    if (mt > -INFINITY) S += tp[(size_t)tt * stride + col + 1] * exp(mt - M);
  }
  S = wave_sum(S);
  return M + log(S);
}
// Block-wide reductions over the 4 waves of a 256-thread block; every thread
// gets the result.  `sh` needs 4 doubles; the leading barrier protects reuse.
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}
__device__ inline double block_max(double v, double* sh) {
  v = wave_max(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

__device__ inline float exp2_hw(float x) { return __builtin_amdgcn_exp2f(x); }

// log2 sum_y 2^w(x, y) of row x from its column-split partials (M_s, S_s),
// M_s the split's max and S_s its sum of 2^(w - M_s); also returns the row max
// M (the next one-pass shift) and the sum S relative to it.
struct Merged { double lse2, M, S; };
__device__ inline Merged merge_splits(const double2* __restrict__ p, int ns) {
  double Mx = -INFINITY;
  for (int s = 0; s < ns; ++s) Mx = fmax(Mx, p[s].x);
  if (!(Mx > -INFINITY)) return {-INFINITY, -INFINITY, 0.0};
  double S = 0.0;
  for (int s = 0; s < ns; ++s) {
    const double2 q = p[s];
    if (q.y > 0.0) S += (q.x == Mx) ? q.y : q.y * exp2(q.x - Mx);
  }
  return {(S > 0.0) ? Mx + log2(S) : -INFINITY, Mx, S};
}
// m_{k->j}(x) in natural log from the column-split partials of row x.
__device__ inline double merge_row(const MsgDesc& md, int x, double x2) {
  const Merged g = merge_splits(md.partial + (size_t)x * md.ns, md.ns);
  return (g.lse2 > -INFINITY) ? kLn2 * g.lse2 - x2 / md.eps : -INFINITY;
}

__device__ inline double sq_norm(const double* xs, int dim, int x) {
  double x2 = 0.0;
  for (int d = 0; d < dim; ++d) x2 = fma(xs[(size_t)x * dim + d], xs[(size_t)x * dim + d], x2);
  return x2;
}

constexpr double kStallGain = 0.97;

// Stop decision of an instance after its half-sweep t, from the stopping sum
// E of the state before the update and its largest per-edge term Em (one
// thread of the instance's finalise block).
__device__ void decide(const Tables& tb, InstState* st, long long t, double E, double Em) {
  bool stop = false;
  if (!isfinite(E)) {
    st->done = kNonFinite;
    if (t >= 2) st->t = t - 1;  // roll back to the last state whose sum was finite
    stop = true;
  } else {
    st->err_sum = E;
    st->err_max = Em;
    st->checked_t = t;
    // progress: a sum at least kStallGain below the last recorded one (a
    // sum jittering at a noise floor sets no new record by chance)
    if (E < kStallGain * st->best_err) {
      st->best_err = E;
      st->best_t = t;
    }
    if (t >= st->min_check_t && E <= st->tol) {
      st->done = kConverged;  // this half-sweep wrote only the unread slots
      stop = true;
    } else if (st->stall_window > 0 && t - st->best_t >= st->stall_window) {
      st->done = kStalled;    // no new minimum for a while: the state before t is kept
      stop = true;
    } else {
      st->t = t + 1;
      st->updates += 1;
      if (st->updates >= st->max_updates) {
        st->done = kMaxSteps;
        stop = true;
      }
    }
  }
  if (stop) {
    st->clk_stop = wall_clock64();
    atomicAdd(tb.ndone, 1);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Evaluation message kernel (FP64, two passes).  Block = 4 waves; lane l of
// wave w owns rows row0 + (w*R + r)*64 + l, r < R; columns stream through LDS
// in chunks.  Per chunk, pass 1 finds the row max and pass 2 sums 2^(w - max);
// the running sum is rescaled when the max grows.  Output per row and column
// split: (M, sum 2^(w - M)), M the split's max, merged by the evaluation node
// pass.  The potentials are read from the given slot of the source class.
// ---------------------------------------------------------------------------
template <int DIM, int R, bool EXPL>
__global__ __launch_bounds__(kBlock) void k_msg(Tables tb, int src_slot) {
  constexpr int CH = EXPL ? 32 : kChunk;            // columns per LDS chunk
  constexpr int STR = EXPL ? 1 : (DIM == 1 ? 2 : 4); // doubles per staged column
  constexpr int TM = 256 * R;                        // rows per block
  __shared__ double s_col[CH * STR];
  __shared__ float s_cost[EXPL ? CH * TM : 1];

  const K1Item it = tb.items[blockIdx.x];
  const MsgDesc* __restrict__ md = tb.msgs + it.msg;
  if (src_slot < 0) src_slot = tb.inst_slot[2 * it.inst + (1 - tb.colour)];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n_dst = md->n_dst;
  const double eps = md->eps;
  const double cxs = 2.0 * kLog2e / eps;
  const double ces = -kLog2e / eps;
  const double* __restrict__ lam = md->lam_src[src_slot];
  const double csrc = md->c_src ? md->c_src[src_slot] : 0.0;
  const double* __restrict__ lg = md->lg_src;
  const double* __restrict__ ys = md->supp_src;

  int row[R];
  double cx[R][DIM];
  double Mrun[R], Srun[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    row[r] = it.row0 + (wave * R + r) * 64 + lane;
    const bool v = row[r] < n_dst;
#pragma unroll
    for (int d = 0; d < DIM; ++d) cx[r][d] = (v && !EXPL) ? cxs * md->supp_dst[(size_t)row[r] * DIM + d] : 0.0;
    Mrun[r] = -INFINITY;
    Srun[r] = 0.0;
  }
  auto wval = [&](int r, int c, double a) -> double {
    double w = a;
    if (EXPL) {
      w = fma(ces, (double)s_cost[c * TM + (wave * R + r) * 64 + lane], w);
    } else {
#pragma unroll
      for (int d = 0; d < DIM; ++d) w = fma(cx[r][d], s_col[c * STR + 1 + d], w);
    }
    return w;
  };

  for (int c0 = 0; c0 < it.ncols; c0 += CH) {
    const int cn = min(CH, it.ncols - c0);
    __syncthreads();  // previous chunk fully consumed
    if (threadIdx.x < cn) {
      const int col = it.col0 + c0 + threadIdx.x;
      double base = (lam[col] - csrc) + lg[col];
      if (!EXPL) {
        double y2 = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const double y = ys[(size_t)col * DIM + d];
          s_col[threadIdx.x * STR + 1 + d] = y;
          y2 = fma(y, y, y2);
        }
        base -= y2 / eps;
      }
      s_col[threadIdx.x * STR] = kLog2e * base;
    }
    if (EXPL) {
      // cost tile, stored src-major: cost[y * n_dst + x]; coalesced over x
      for (int c = 0; c < cn; ++c) {
        const int col = it.col0 + c0 + c;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int lr = r * 256 + threadIdx.x;
          const int x = it.row0 + lr;
          s_cost[c * TM + lr] = x < n_dst ? md->cost[(size_t)col * n_dst + x] : 0.0f;
        }
      }
    }
    __syncthreads();
    double Mc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) Mc[r] = -INFINITY;
    for (int c = 0; c < cn; ++c) {
      const double a = s_col[c * STR];
#pragma unroll
      for (int r = 0; r < R; ++r) Mc[r] = fmax(Mc[r], wval(r, c, a));
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (Mc[r] > Mrun[r]) {
        Srun[r] *= exp2(Mrun[r] - Mc[r]);  // 0 when Mrun = -inf and Srun = 0
        Mrun[r] = Mc[r];
      }
      const double sh = (Mrun[r] == -INFINITY) ? 0.0 : Mrun[r];
      double S = 0.0;
      for (int c = 0; c < cn; ++c) S += exp2(wval(r, c, s_col[c * STR]) - sh);
      Srun[r] += S;
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (row[r] < n_dst) md->partial[(size_t)row[r] * md->ns + it.split] = make_double2(Mrun[r], Srun[r]);
  }
}

// ---------------------------------------------------------------------------
// Node kernel: one half-sweep's work for one 64-row tile of a node j of the
// class being updated (Algorithm tree_local_reg; one lane per row x).
//
//   messages  for every incident edge (j, k), m_{k->j}(x) = LSE over supp(k):
//             the W waves of the block split supp(k) into W column ranges; each
//             wave streams its range through its own LDS staging buffer and
//             returns (max, sum 2^(w - max)) per row; the partials are merged
//             in FP64 through LDS by one wave per edge (edges rotate over the
//             waves, so merging overlaps the next edge's sums).
//   terms     of the state before the update (Lemma f_upper_bound_tree):
//             fixed: mu(x) |expm1(Lam_(j,k)(x) + m_{k->j}(x))| = |q_(j,k)(x) - mu(x)|,
//             free:  |q_(j,k)(x) - qbar(x)|, q = exp(Lam + m), qbar the mean over k
//   update    (eq. bipartite_tree_updates1/2 in the closed form of Prop. equi)
//             fixed: L_(j,k) = -m_{k->j}; free: L_(j,k) = abar - m_{k->j},
//             abar = mean_k m_{k->j}, with the normaliser c_j = LSE_x abar formed
//             by the finalise kernel from the tile records.
//   record    per edge the tile's sum of terms, then (max, scaled sum) of abar.
//
// Sums (FP32 core): pairs of v_exp_f32 terms of the FP64-reduced argument,
// added in FP32 and accumulated in FP64.  From the third half-sweep of a call
// on, one pass shifted by the previous max of the same row and column range
// (kept in wmax: the log2 of the largest FP32 pair sum, so the max term to
// within one binade above it), tracked alongside as the max of the pair sums;
// a chunk whose sum exceeds 2^kShiftHi (so a term may have overflowed) moves
// the shift to its exact max and is summed again, and a row whose sum ends
// below 2^kShiftLo (terms may have underflowed) sends the wave back through
// its range in two passes.  Both decisions are wave-uniform.
// The first two half-sweeps of a call take two passes (chunk max, then sum);
// the FP64 variant (F64) always does, with FP64 exponentials.
// ---------------------------------------------------------------------------
// Global address space views of device arrays reached through descriptors:
// loads through them are counted in order with the other vector loads, so a
// prefetch does not force a wait at the end of its (divergent) block.
typedef const __attribute__((address_space(1))) double GDbl;
typedef __attribute__((address_space(1))) double GDblW;
typedef const __attribute__((address_space(1))) float GFlt;
// Message descriptors are written only by the host, between launches: read
// through the constant address space, a wave-uniform descriptor field is one
// scalar load instead of a vector load per lane.
typedef const __attribute__((address_space(4))) MsgDesc CMsg;
constexpr int kFinWaves = 16;    // waves per finalise block (one node each)
constexpr double kShiftHi = 96.0;
constexpr double kShiftLo = -96.0;
constexpr double kSumHi = 0x1p96;   // 2^kShiftHi
constexpr double kSumLo = 0x1p-96;  // 2^kShiftLo
constexpr int kNodeDegLDS = 16;  // merged messages of the first 16 edges stay in LDS

// The finalise step of one instance (one block of NW waves, one wave per node
// of the class, nodes w, w + NW, ...): per-edge terms summed over the node's
// tile records (lanes over tiles), every free node's normaliser c_j = LSE over
// its tile records of abar, then the terms summed in a fixed order and the stop
// decision by thread 0.  `colour` is the class whose records are complete; the
// step does nothing unless the instance's next undecided half-sweep is of that
// class.  It then publishes the view read by later node launches: run separately
// after a node launch (fused = false) for the next two launches; carried by the
// next node launch (fused = true), only for the launch after it, since that
// launch's own node blocks are reading the other view.
// The stopping sum is accumulated in kFinParts partial sums (node i into part
// i mod kFinParts) added in part order, so it does not depend on NW.
constexpr int kFinParts = 16;
constexpr int kFinEdges = 2;  // edges whose record entries a finalise wave loads together

template <int NW>
__device__ void fin_instance(const Tables& tb, const NodeItem* __restrict__ nodes, int colour, InstState* st,
                             bool fused, double (*sh)[2]) {
  static_assert(kFinParts % NW == 0, "each wave takes whole parts");
  constexpr int Q = kFinParts / NW;  // parts per wave: wv, wv + NW, ...
  const int other = 1 - colour;
  if (st->done) {
    if (threadIdx.x == 0) {
      st->vdone[colour] = 1;
      if (!fused) st->vdone[other] = 1;
    }
    return;
  }
  const long long t = st->t;
  if (((t & 1) == 1) != (colour == 0)) return;
  const int nxt = (int)((((t - 1) >> 1) + 1) % kSlots);
  const int i0 = st->node0[colour], cnt = st->nnodes[colour];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double esum[Q], emax = 0.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) esum[q] = 0.0;
  for (int i = wv; i < cnt; i += NW) {
    const NodeItem nd = nodes[i0 + i];
    const int q = (i / NW) % Q;  // node i is in part i mod kFinParts = wv + q * NW
    const int deg = nd.deg, stride = deg + kRecExtra, tiles = nd.tiles;
    const double* __restrict__ tp = nd.tpart;
    // edges k0 .. k0 + 7 at a time: each lane loads those entries of its
    // tiles' records before any reduction, so a node waits for memory once
    // per eight edges; per edge the sum over tiles (lane partials in tile
    // order, then the wave sum) and the order over edges are as one at a time
    for (int k0 = 0; k0 < deg; k0 += kFinEdges) {
      double acc[kFinEdges];
#pragma unroll
      for (int kk = 0; kk < kFinEdges; ++kk) acc[kk] = 0.0;
      for (int tt = lane; tt < tiles; tt += 64) {
#pragma unroll
        for (int kk = 0; kk < kFinEdges; ++kk)
          if (k0 + kk < deg) acc[kk] += tp[(size_t)tt * stride + k0 + kk];
      }
#pragma unroll
      for (int kk = 0; kk < kFinEdges; ++kk) {
        if (k0 + kk < deg) {
          const double e = wave_sum(acc[kk]);
#pragma unroll
          for (int qq = 0; qq < Q; ++qq)
            if (qq == q) esum[qq] += e;
          emax = fmax(emax, e);
        }
      }
    }
    if (!nd.fixed) {
      const int t0 = min(lane, tiles - 1);
      const double c = tile_lse(tp, tiles, stride, deg, tp[(size_t)t0 * stride + deg], tp[(size_t)t0 * stride + deg + 1]);
      if (lane == 0) nd.c[nxt] = c;
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      sh[wv + q * NW][0] = esum[q];
      sh[wv + q * NW][1] = emax;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double E = 0.0, Em = 0.0;
    for (int w = 0; w < kFinParts; ++w) {
      E += sh[w][0];
      Em = fmax(Em, sh[w][1]);
    }
    decide(tb, st, t, E, Em);
    const int stop = st->done != kRunning;
    st->vt[colour] = t + 2;
    st->vdone[colour] = stop;
    if (!fused) {
      st->vt[other] = t + 1;
      st->vdone[other] = stop;
    }
  }
}

// Orders a wave's LDS writes before its later LDS reads (wave-private buffers).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int DIM, int W, int R, int H, bool F64, bool EXPL>
// The 8-wave, 32-row-tile shape asks for four waves per SIMD (at most 128
// VGPRs), so that two of its blocks share a CU; so does the one-row-per-lane
// FP32-core shape of one-dimensional supports (otherwise one VGPR over 128,
// and three waves per SIMD).
__global__ __launch_bounds__(64 * W, ((W == 8 && R == 1 && H == 2 && !EXPL) ||
                                      (DIM == 1 && R == 1 && H == 1 && !EXPL && !F64)) ? 4 : 1)
void k_node(Tables tb) {
  static_assert(H == 1 || !EXPL, "explicit costs take one lane group");
  constexpr int LPR = 64 / H;                        // lanes per lane group
  constexpr int CH = EXPL ? 32 : 64;                 // columns per wave chunk
  constexpr int CHH = CH / H;                        // columns per lane-group chunk
  constexpr int STR = EXPL ? 1 : (DIM == 1 ? 2 : 4); // doubles per staged column
  constexpr int TR = LPR * R;                        // rows per tile
  constexpr int NT = 64 * W;                         // threads per block
  // one-dimensional on-the-fly costs fold an affine part of the one-pass
  // shift into the staged columns (one FP64 FMA per pair)
  constexpr bool FOLD = DIM == 1 && !EXPL && !F64;
  // (edge, range) partials: deg * H ranges when deg >= W (deg <= kNodeDegLDS), else W * H
  constexpr int NP = (kNodeDegLDS > W ? kNodeDegLDS : W) * H;
  __shared__ double s_col[W][CH * STR];
  __shared__ double2 s_part[NP][TR];  // (edge, range) partials; then per-(edge, row) terms
  __shared__ double s_m[kNodeDegLDS][TR];
  __shared__ double s_l[kNodeDegLDS][TR];  // held L_(j,k)(x) of the update phase
  __shared__ double s_mu[TR];
  __shared__ double s_x2[TR];
  __shared__ double s_csrc[kNodeDegLDS];  // c_k of each edge's source node

  if ((int)blockIdx.x < tb.n_fin) {
    // the finalise step of the previous launch's half-sweep, one block per instance
    __shared__ double sh_fin[kFinParts][2];
    fin_instance<W>(tb, tb.fin_nodes, tb.fin_colour, tb.inst + blockIdx.x, true, sh_fin);
    return;
  }
  const TileItem ti = tb.tiles[blockIdx.x - tb.n_fin];
  const InstState* st = tb.inst + ti.inst;
  const NodeItem nd = tb.nodes[ti.node];
  const CMsg* __restrict__ mds = (const CMsg*)(tb.msgs + ti.msg0);
  const int n = ti.n, deg = ti.deg;
  // the wave index is the same on every lane; said so, the edge it picks and
  // that edge's descriptor reads are wave-uniform
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  // H lane groups of LPR lanes: lane (group h, index i) holds rows i, i + LPR, ...
  // of the tile and sums column range h of its wave's share of each edge
  const int lrow = lane % LPR, half = lane / LPR;
  // Edges run on different waves: with deg >= W each wave takes whole edges
  // (k = wv, wv + W, ...); otherwise g = W / deg waves share an edge.  Each
  // wave's share is split over its H lane groups: gr = g * H column ranges per
  // edge, range rid = sub * H + half.
  const int g = deg >= W ? 1 : W / deg;
  const int gr = g * H;
  const int k_first = deg >= W ? wv : (wv < deg * g ? wv / g : deg);
  const int k_step = deg >= W ? W : deg;
  const int sub = deg >= W ? 0 : wv % g;
  // The first chunk of the wave's first edge (log gamma and supports) and
  // that edge's stored shifts, loaded before the instance state arrives: none
  // of it depends on the half-sweep (the source potentials do, through their
  // slot, and are read after the state check; reading all three slots here
  // was slower).  A wave without an edge reads the last edge's and ignores
  // them.
  const int kp = min(k_first, deg - 1);
  const int p_nsrc = mds[kp].n_src, p_rid = sub * H + half;
  const int p_col = min(min(p_rid * ((p_nsrc + gr - 1) / gr), p_nsrc) + lrow, p_nsrc - 1);
  double pf_y[DIM > 0 ? DIM : 1], pf_pm[R];
  const double pf_g = ((const GDbl*)mds[kp].lg_src)[p_col];
#pragma unroll
  for (int d = 0; d < DIM; ++d) pf_y[d] = EXPL ? 0.0 : ((const GDbl*)mds[kp].supp_src)[(size_t)p_col * DIM + d];
#pragma unroll
  for (int r = 0; r < R; ++r)
    pf_pm[r] = ((const GDbl*)mds[kp].wmax)[(size_t)p_rid * n + min(ti.row0 + r * LPR + lrow, n - 1)];
  // this thread's rows' supports (clamped: unconditional loads)
  double pf_x[R][DIM > 0 ? DIM : 1];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int d = 0; d < DIM; ++d)
      pf_x[r][d] = EXPL ? 0.0 : ((const GDbl*)mds[0].supp_dst)[(size_t)min(ti.row0 + r * LPR + lrow, n - 1) * DIM + d];
  // the instance's view of the loop state (scalar loads, issued with the above)
  const long long t = st->vt[tb.colour];
  const bool inst_done = st->vdone[tb.colour] != 0;
  const long long t_first = st->t_first, onepass_from = st->onepass_from;
  // keeps every load above here: without it the column loads sink below the
  // state check (their values are used only after it)
  asm volatile("" ::: "memory");
  if (inst_done || t < t_first || ((t & 1) == 1) != (tb.colour == 0)) return;
  // slots: this class's held state before t, its update, the other class's held state
  const int cur = (int)(((t - 1) >> 1) % kSlots), nxt = (cur + 1) % kSlots;
  const int src_slot = (int)((t >> 1) % kSlots);
  const bool one = !F64 && t >= onepass_from;
  const bool rec_ok = t - 1 >= t_first;
  const bool lds = deg <= kNodeDegLDS;
  const bool fixed = ti.fixed != 0;
  int x[R];
  bool vx[R];
  const double eps = mds[0].eps;
  const double cxs = 2.0 * kLog2e / eps;
  const double ces = -kLog2e / eps;
  double cx[R][DIM > 0 ? DIM : 1];
  double x2[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    x[r] = ti.row0 + r * LPR + lrow;
    vx[r] = x[r] < n;
    x2[r] = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double v = (vx[r] && !EXPL) ? pf_x[r][d] : 0.0;
      cx[r][d] = cxs * v;
      x2[r] = fma(v, v, x2[r]);
    }
  }
  double* __restrict__ stage = s_col[wv];
  // the held potential (and mu) of this thread's first (edge, row) item of the
  // update phase, loaded now so that phase does not wait for memory
  // (unconditional loads at clamped indexes, so the waits before the column
  // loop can count them; the values of threads without an item are unused)
  double l_item, mu_item;
  {
    const int k = min((int)threadIdx.x / TR, deg - 1);
    const int xr = min(ti.row0 + (int)threadIdx.x - k * TR, n - 1);
    l_item = ((const GDbl*)mds[k].lam_dst[cur])[xr];
    const double mv = ((const GDbl*)(fixed ? nd.mu : mds[k].lam_dst[cur]))[xr];
    mu_item = fixed ? mv : 0.0;
  }
  // this node's held normaliser (free nodes; a constrained node has no slots
  // and reads any valid address), needed by the update phase
  const double c_held_j = *(const GDbl*)(nd.c ? nd.c + cur : mds[0].lam_dst[0]);

  // One edge's sums.  LDS_T: the partials stay in LDS (deg <= kNodeDegLDS);
  // otherwise the message goes to global memory at once.  The two cases are
  // separate loops so the common one holds no global store (a store in flight
  // makes every later wait for a load wait for all of them).
  // PRE: the wave's first edge, whose first chunk and shifts were loaded at entry.
  auto edge_sums = [&](const int k, auto lds_t, auto pre_t) {
    constexpr bool LDS_T = decltype(lds_t)::value;
    constexpr bool PRE = decltype(pre_t)::value;
    const CMsg& md = mds[k];
    const int n_src = md.n_src;
    const int per = (n_src + gr - 1) / gr;
    const int rid = sub * H + half;
    const int c_lo = min(rid * per, n_src), c_hi = min(c_lo + per, n_src);
    // chunk loop length, the same for every lane group (a short last range
    // runs on with empty chunks)
    const int span = H == 1 ? c_hi - c_lo : per;
    // The source's normaliser c_k only shifts the message (m = m' - c_k with m'
    // summed over L + log gamma): it is formed from the source node's tile
    // records (or read from its stored slot) after the column loop.  Every
    // field and value it needs is read here, before the loop: the loop's wave
    // fences would otherwise make the compiler read the descriptor again after
    // it, a chain of dependent loads with nothing to overlap them.
    const GDbl* __restrict__ srec = (const GDbl*)md.src_tpart;
    const int src_deg = md.src_deg, src_tiles = md.src_tiles;
    const bool src_free = md.src_free != 0;
    const int s_stride = src_deg + kRecExtra, s_tile = min(lane, src_tiles - 1);
    const double rec_m0 = srec[(size_t)s_tile * s_stride + src_deg];
    const double rec_s0 = srec[(size_t)s_tile * s_stride + src_deg + 1];
    // a constrained source has no slots (c = 0); the load then reads any valid
    // address and its value is not used
    const double c_held = *(const GDbl*)(md.c_src ? md.c_src + src_slot : md.lam_src[src_slot]);
    const GDbl* __restrict__ lam = (const GDbl*)md.lam_src[src_slot];
    const GDbl* __restrict__ lg = (const GDbl*)md.lg_src;
    const GDbl* __restrict__ ys = (const GDbl*)md.supp_src;
    const GFlt* __restrict__ cost = (const GFlt*)md.cost_tile;
    GDblW* __restrict__ wmax = (GDblW*)md.wmax;

    // A chunk's column data is fetched into registers (lane = column of its
    // group's range), then staged in the wave's LDS buffer (group h at column
    // h * CHH); padded columns get a = -inf and y = 0, so they add exactly
    // nothing.  The one-pass loop fetches the next chunk before summing the
    // current one, so its loads overlap the arithmetic.
    // staged columns are (a(y) - al, y - be): al = be = 0 except in the
    // one-pass sums of FOLD kernels
    double al = 0.0, be = 0.0;
    // A fetch only issues the loads (lane lrow: column c0 + lrow, clamped into
    // the support, with a flag for columns inside the chunk); all arithmetic
    // on them happens at staging, so loads of later chunks stay in flight.
    struct Raw {
      double l, g, y[DIM > 0 ? DIM : 1];
      bool v;
    };
    Raw f_raw, g_raw;
    auto fetch_into = [&](int c0, int cn, Raw& o) {
      const int col = min(c0 + lrow, n_src - 1);
      o.v = lrow < cn;
      o.l = lam[col];
      o.g = lg[col];
      if (!EXPL) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) o.y[d] = ys[(size_t)col * DIM + d];
      }
    };
    auto fetch_chunk = [&](int c0, int cn) { fetch_into(c0, cn, f_raw); };
    // the chunk after next goes to the second register set; move it up
    auto advance = [&]() { f_raw = g_raw; };
    auto stage_fetched = [&]() {
      double a = -INFINITY, yv[DIM > 0 ? DIM : 1];
#pragma unroll
      for (int d = 0; d < DIM; ++d) yv[d] = 0.0;
      if (f_raw.v) {
        a = f_raw.l + f_raw.g;
        if (!EXPL) {
          double y2 = 0.0;
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            yv[d] = f_raw.y[d];
            y2 = fma(yv[d], yv[d], y2);
          }
          a -= y2 / eps;
        }
        a = a * kLog2e - al;
      }
      if (lrow < CHH) {
        const int sc = (half * CHH + lrow) * STR;
        stage[sc] = a;
        if (!EXPL) {
#pragma unroll
          for (int d = 0; d < DIM; ++d) stage[sc + 1 + d] = yv[d] - (d == 0 ? be : 0.0);
        }
      }
      wave_sync();
    };
    auto stage_chunk = [&](int c0, int cn) {
      fetch_chunk(c0, cn);
      stage_fetched();
    };
    const double* __restrict__ sth = stage + half * CHH * STR;  // this lane group's columns
    // explicit costs (tile-major: a wave's chunk is one contiguous 8 KB run):
    // cv holds the chunk being summed, cq the next one's, loaded a chunk ahead
    // (columns clamped into the matrix, past the range they meet a = -inf;
    // rows past n read the zero padding and are never used)
    float cv[EXPL ? R : 1][EXPL ? CH : 1], cq[EXPL ? R : 1][EXPL ? CH : 1];
    auto fetch_cost = [&](int c0) {
      if (EXPL) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int c = 0; c < CH; ++c)
            cq[r][c] = cost[((size_t)(x[r] >> 6) * n_src + min(c0 + c, n_src - 1)) * 64 + (x[r] & 63)];
      }
    };
    auto take_cost = [&]() {
      if (EXPL) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int c = 0; c < CH; ++c) cv[r][c] = cq[r][c];
      }
    };
    auto load_cost = [&](int c0, int) {
      fetch_cost(c0);
      take_cost();
    };
    auto wcol = [&](int r, int c, double a) -> double {
      double w = a;
      if (EXPL) {
        w = fma(ces, (double)cv[r][c], w);
      } else {
#pragma unroll
        for (int d = 0; d < DIM; ++d) w = fma(cx[r][d], sth[c * STR + 1 + d], w);
      }
      return w;
    };
    // sums of 2^(w - sh[r]) over the staged chunk (padded columns give 0)
    auto chunk_sum = [&](const double* sh, double* Sc) {
#pragma unroll
      for (int r = 0; r < R; ++r) Sc[r] = 0.0;
#pragma unroll 4
      for (int c = 0; c < CHH; c += 2) {
        const double a0 = sth[c * STR], a1 = sth[(c + 1) * STR];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double w0 = wcol(r, c, a0), w1 = wcol(r, c + 1, a1);
          if (F64) {
            Sc[r] += exp2(w0 - sh[r]) + exp2(w1 - sh[r]);
          } else {
            const float p = exp2_hw((float)(w0 - sh[r])) + exp2_hw((float)(w1 - sh[r]));
            Sc[r] += (double)p;
          }
        }
      }
    };
    // maxima over the staged chunk of the staged exponent minus off[r]
    auto chunk_max = [&](const double* off, double* Mc) {
#pragma unroll
      for (int r = 0; r < R; ++r) Mc[r] = -INFINITY;
#pragma unroll 4
      for (int c = 0; c < CHH; ++c) {
        const double a = sth[c * STR];
#pragma unroll
        for (int r = 0; r < R; ++r) Mc[r] = fmax(Mc[r], wcol(r, c, a) - off[r]);
      }
    };

    double M[R], S[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      M[r] = -INFINITY;
      S[r] = 0.0;
    }
    bool two = !one;
    if (one) {
      // Row x is shifted by s(x) = sb(x) + dl(x).  With FOLD, sb(x) = al + be cx(x)
      // is the chord, over the lane group's rows of least and greatest cx, of the
      // previous row shifts (maxima of exponents affine in cx, so convex in
      // cx), folded into the staged columns; a wave whose every row's previous
      // shift lies within [-64, 32] of the chord sums with dl = 0 and one FMA
      // per pair ("folded"), otherwise (and after a re-shift) dl(x) carries the
      // rest of the previous shift ("row mode").  Without FOLD, sb = 0 and s(x)
      // is the previous shift as is.
      double sb[R], dl[R];
      bool pmok[R];
      double pmv[R];
      // Every load here is unconditional (indexes clamped into the arrays), so
      // the compiler can wait for exactly the ones a step needs: the previous
      // maxima first, then the first two chunks' columns (only their staging
      // needs the shift).
#pragma unroll
      for (int r = 0; r < R; ++r) {
        pmv[r] = PRE ? pf_pm[r] : (double)wmax[(size_t)rid * n + min(x[r], n - 1)];
        sb[r] = 0.0;
      }
      if constexpr (PRE) {
        // the column fetch_chunk(c_lo, ...) would load, in the current slot
        f_raw.v = lrow < min(CHH, c_hi - c_lo);
        f_raw.l = lam[p_col];
        f_raw.g = pf_g;
#pragma unroll
        for (int d = 0; d < DIM; ++d) f_raw.y[d] = pf_y[d];
      } else {
        fetch_chunk(c_lo, min(CHH, c_hi - c_lo));
      }
      fetch_into(c_lo + CHH, min(CHH, c_hi - c_lo - CHH), g_raw);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!vx[r]) pmv[r] = 0.0;
        pmok[r] = vx[r] && isfinite(pmv[r]);
      }
      bool rowmode = true;
      if constexpr (FOLD) {
        // chord through the lane group's first and last valid rows (the rows
        // of least and greatest cx when the supports are sorted; otherwise the
        // check below sends the wave to row mode), read with v_readlane
        const int i_last = min(TR, n - ti.row0) - 1;  // >= 0: the tile has a valid row
        const int r_last = i_last / LPR, l_last = i_last - r_last * LPR;
        double cl = 0.0, pl = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (r == r_last) {
            cl = cx[r][0];
            pl = pmv[r];
          }
        auto rdl = [](double v, int l) -> double {
          const long long b = __double_as_longlong(v);
          const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
          const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
          return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
        };
        double c0v = rdl(cx[0][0], 0), p0v = rdl(pmv[0], 0), c1v = rdl(cl, l_last), p1v = rdl(pl, l_last);
        if (H == 2) {
          const double c0h = rdl(cx[0][0], LPR), p0h = rdl(pmv[0], LPR);
          const double c1h = rdl(cl, LPR + l_last), p1h = rdl(pl, LPR + l_last);
          if (half) {
            c0v = c0h; p0v = p0h; c1v = c1h; p1v = p1h;
          }
        }
        if (isfinite(p0v) && isfinite(p1v)) {
          if (c1v != c0v) {
            be = (p1v - p0v) / (c1v - c0v);
            al = p0v - be * c0v;
          } else {
            al = fmax(p0v, p1v);
          }
        }
        if (!isfinite(al) || !isfinite(be)) al = be = 0.0;
        int bad = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          sb[r] = fma(be, cx[r][0], al);
          if (pmok[r] && !(pmv[r] - sb[r] >= -64.0 && pmv[r] - sb[r] <= 32.0)) bad = 1;
        }
        rowmode = __any(bad);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) dl[r] = rowmode ? (pmok[r] ? pmv[r] : 0.0) - sb[r] : 0.0;

      float Mp[R];  // max pair sum relative to the shift, over the range
#pragma unroll
      for (int r = 0; r < R; ++r) Mp[r] = 0.0f;
      fetch_cost(c_lo);
      for (int j0 = 0; j0 < span; j0 += CHH) {
        const int c0 = c_lo + j0;
        take_cost();
        stage_fetched();
        advance();
        fetch_into(c0 + 2 * CHH, min(CHH, c_hi - c0 - 2 * CHH), g_raw);  // past the range: masked
        fetch_cost(c0 + CHH);
        // one pass: sums of 2^(d) with d the staged exponent minus dl, and
        // the max of the FP32 pair sums (within a factor 2 of the max term)
        double Sc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) Sc[r] = 0.0;
        auto pass = [&](auto row_t) {
          constexpr bool ROW = decltype(row_t)::value;
#pragma unroll 4
          for (int c = 0; c < CHH; c += 2) {
            const double a0 = sth[c * STR], a1 = sth[(c + 1) * STR];
#pragma unroll
            for (int r = 0; r < R; ++r) {
              double d0 = wcol(r, c, a0), d1 = wcol(r, c + 1, a1);
              if (ROW) {
                d0 -= dl[r];
                d1 -= dl[r];
              }
              const float p = exp2_hw((float)d0) + exp2_hw((float)d1);
              Mp[r] = fmaxf(Mp[r], p);
              Sc[r] += (double)p;
            }
          }
        };
        if (rowmode) pass(std::true_type{});
        else pass(std::false_type{});
        // The terms are positive, so a chunk sum within 2^kShiftHi bounds every
        // term (an FP32 overflow gives inf and fails the test too)
        int hi = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) hi |= (vx[r] && !(Sc[r] <= kSumHi)) ? 1 : 0;
        if (__any(hi)) {
          // exact FP64 maxima; rows far above their shift move it and the
          // chunk is summed again in row mode
          double Md[R];
          chunk_max(dl, Md);
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if (Md[r] > kShiftHi) {
              // this chunk's max term is now 2^0, above every earlier one
              S[r] *= exp2(-Md[r]);
              dl[r] += Md[r];
              Mp[r] = 1.0f;
            }
          }
          rowmode = true;
          chunk_sum(dl, Sc);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) S[r] += Sc[r];
        wave_sync();
      }
      // A row of a non-empty range whose sum ends below 2^kShiftLo may have
      // lost terms to FP32 underflow (or has no finite term): two passes.
      // Otherwise the range reports M = shift + log2 of its largest pair sum
      // (the max term to within one binade, the next shift) and S relative
      // to M; M + log2 S is the shift plus log2 of the sum, whatever the
      // rounding of the FP32 log.
      int lo = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) lo |= (vx[r] && c_hi > c_lo && !(S[r] >= kSumLo)) ? 1 : 0;
      if (__any(lo)) {
        two = true;
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (S[r] > 0.0) {
            const double lm = (double)__builtin_amdgcn_logf(Mp[r]);
            M[r] = (sb[r] + dl[r]) + lm;
            S[r] *= exp2(-lm);
          } else {
            M[r] = -INFINITY;
          }
        }
      }
    }
    if (two) {
      al = be = 0.0;
      const double zero[R] = {};
#pragma unroll
      for (int r = 0; r < R; ++r) {
        M[r] = -INFINITY;
        S[r] = 0.0;
      }
      for (int j0 = 0; j0 < span; j0 += CHH) {
        const int c0 = c_lo + j0;
        const int cn = min(CHH, c_hi - c0);
        load_cost(c0, cn);
        stage_chunk(c0, cn);
        double Mc[R], Sc[R], sh[R];
        chunk_max(zero, Mc);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (Mc[r] > M[r]) {
            S[r] *= exp2(M[r] - Mc[r]);  // 0 when M = -inf and S = 0
            M[r] = Mc[r];
          }
          sh[r] = M[r] == -INFINITY ? 0.0 : M[r];
        }
        chunk_sum(sh, Sc);
#pragma unroll
        for (int r = 0; r < R; ++r) S[r] += Sc[r];
        wave_sync();
      }
    }
    // from the records when the source's last update (half-sweep t - 1) ran in
    // this run, else its stored normaliser
    double ck = 0.0;
    if (sub == 0 && src_free)
      ck = rec_ok ? tile_lse((const double*)srec, src_tiles, s_stride, src_deg, rec_m0, rec_s0) : c_held;
    if (LDS_T && sub == 0 && lane == 0) s_csrc[k] = ck;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (LDS_T) {
        // the ranges' next shifts go to wmax after the merge below
        s_part[k * gr + rid][r * LPR + lrow] = make_double2(M[r], S[r]);
      } else {
        if (vx[r]) wmax[(size_t)rid * n + x[r]] = M[r];
        // one wave per edge (g = 1): its H ranges merged across the lane
        // groups, the message goes straight to mfull
        double Mm = M[r], Sm = S[r];
        if (H == 2) {
          const double Mo = __shfl_xor(Mm, LPR), So = __shfl_xor(Sm, LPR);
          const double Mx = fmax(Mm, Mo);
          double St = 0.0;
          if (Mx > -INFINITY) {
            if (Sm > 0.0) St += Sm * exp2(Mm - Mx);
            if (So > 0.0) St += So * exp2(Mo - Mx);
          }
          Mm = Mx;
          Sm = St;
        }
        if (vx[r] && half == 0)
          md.mfull[x[r]] = (Mm > -INFINITY && Sm > 0.0) ? kLn2 * (Mm + log2(Sm)) - x2[r] / eps - ck : -INFINITY;
      }
    }
  };
  if (lds) {
    if (k_first < deg) edge_sums(k_first, std::true_type{}, std::true_type{});
    for (int k = k_first + k_step; k < deg; k += k_step) edge_sums(k, std::true_type{}, std::false_type{});
    // |x|^2 of the tile's rows for the merge (written here, not at entry, so
    // that no wait for the entry loads comes before the column loop)
    if (wv == 0 && half == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) s_x2[r * LPR + lrow] = x2[r];
    }
    // the held potentials and mu of every (edge, row) into LDS for the row
    // owners below (the first item's were loaded at entry)
    for (int it = threadIdx.x; it < deg * TR; it += NT) {
      const int k = it / TR, lr = it - k * TR, xr = ti.row0 + lr;
      double l = l_item, mu = mu_item;
      if (it != (int)threadIdx.x && xr < n) {
        l = mds[k].lam_dst[cur][xr];
        if (fixed && k == 0) mu = nd.mu[xr];
      }
      s_l[k][lr] = l;
      if (k == 0) s_mu[lr] = mu;
    }
  } else {
    if (k_first < deg) edge_sums(k_first, std::false_type{}, std::true_type{});
    for (int k = k_first + k_step; k < deg; k += k_step) edge_sums(k, std::false_type{}, std::false_type{});
  }
  __syncthreads();
  constexpr int RR = TR < 64 ? TR : 64;  // rows per tile record
  constexpr int TQ = TR / RR;            // records per tile
  const double c_old = nd.c ? c_held_j : 0.0;
  // a message-only item (one edge of a node whose update runs in k_node_sep)
  const bool msg_only = ti.msg_only != 0;

  if (lds) {
    // merge the gr ranges of every (edge, row) into m (natural log).  With
    // four ranges or more (QL = 4), four lanes per (edge, row), lane q taking
    // ranges q, q + 4, ..., their max and rescaled sums combined over the quad
    // with DPP (a quad is always active as a whole: the loop bound and NT are
    // multiples of four); with fewer (whole edges per wave), one lane each.
    const int QL = gr >= 4 ? 4 : 1;
    for (int it = threadIdx.x; it < deg * TR * QL; it += NT) {
      const int item = QL == 4 ? it >> 2 : it, q = QL == 4 ? it & 3 : 0;
      const int k = item / TR, lr = item - k * TR;
      double Mq = -INFINITY;
      for (int u = q; u < gr; u += QL) Mq = fmax(Mq, s_part[k * gr + u][lr].x);
      double Mx = Mq;
      if (QL == 4) {
        Mx = fmax(Mx, dpp_move<kDppXor1>(Mx));
        Mx = fmax(Mx, dpp_move<kDppXor2>(Mx));
      }
      double Sq = 0.0;
      if (Mx > -INFINITY) {
        for (int u = q; u < gr; u += QL) {
          const double2 e = s_part[k * gr + u][lr];
          if (e.y > 0.0) Sq += (e.x == Mx) ? e.y : e.y * exp2(e.x - Mx);
        }
      }
      double St = Sq;
      if (QL == 4) {
        St += dpp_move<kDppXor1>(St);
        St += dpp_move<kDppXor2>(St);
      }
      if (q == 0)
        s_m[k][lr] = (Mx > -INFINITY && St > 0.0) ? kLn2 * (Mx + log2(St)) - s_x2[lr] / eps - s_csrc[k] : -INFINITY;
    }
    __syncthreads();
    // Each range's M (its max, or within one binade above it) is the row's
    // next one-pass shift; it stays in s_part (.x) until stored here, after
    // the merge: a store in flight would make the row owners' next wait for
    // a load wait for the store's completion too.  Waves that own no rows
    // store them while the owners work; with no such wave (two waves over
    // 128-row tiles), every thread does so at its end.
    constexpr bool SPARE = W > TQ;
    auto store_shifts = [&](int t0, int stride) {
      for (int it = t0; it < deg * gr * TR; it += stride) {
        const int ku = it / TR, lr = it - ku * TR, k = ku / gr, u = ku - k * gr;
        const int xr = ti.row0 + lr;
        if (xr < n) ((GDblW*)mds[k].wmax)[(size_t)u * n + xr] = s_part[ku][lr].x;
      }
    };
    if (msg_only) {
      // the messages go to mfull for the update kernel, with the next shifts
      for (int it = threadIdx.x; it < deg * TR; it += NT) {
        const int k = it / TR, lr = it - k * TR, xr = ti.row0 + lr;
        if (xr < n) ((GDblW*)mds[k].mfull)[xr] = s_m[k][lr];
      }
      store_shifts(threadIdx.x, NT);
      return;
    }
    // Row owners: wave q takes rows q * RR + lane of the tile and, for each
    // row, every edge in order (terms of the state before the update, the
    // update), then sums its 64 rows into the row block's record: per edge the
    // terms, then (max, scaled sum) of abar.  No block barrier after the merge.
    if (wv >= TQ) {
      store_shifts((wv - TQ) * 64 + lane, (W - TQ) * 64);
      return;
    }
    if (ti.row0 + wv * RR >= n) {
      if (!SPARE) store_shifts(threadIdx.x, NT);
      return;
    }
    const int lr = wv * RR + (lane < RR ? lane : 0), xr = ti.row0 + lr;
    const bool vr = lane < RR && xr < n;  // lanes past RR (RR = 32) only join the sums
    // global-space stores: a flat store also counts as an LDS access, so the
    // next edge's LDS reads would wait for it to complete
    GDblW* __restrict__ rec = (GDblW*)(nd.tpart + (size_t)(ti.row0 / RR + wv) * (deg + kRecExtra));
    if (fixed) {
      const double mu = s_mu[lr];
      for (int k = 0; k < deg; ++k) {
        const double m = s_m[k][lr];
        double term = 0.0;
        if (vr) {
          if (mu > 0.0) term = mu * fabs(expm1(s_l[k][lr] + m));
          ((GDblW*)mds[k].lam_dst[nxt])[xr] = -m;
        }
        term = wave_sum(term);
        if (lane == 0) rec[k] = term;
      }
    } else {
      double as = 0.0, qs = 0.0;
      for (int k = 0; k < deg; ++k) {
        const double m = s_m[k][lr];
        const double q = vr ? exp(s_l[k][lr] - c_old + m) : 0.0;
        if (lane < RR) s_part[k][lr].y = q;  // this lane's own scratch from here on
        as += m;
        qs += q;
      }
      const double ab = as / deg, qb = qs / deg;
      for (int k = 0; k < deg; ++k) {
        double term = 0.0;
        if (vr) {
          term = fabs(s_part[k][lr].y - qb);
          ((GDblW*)mds[k].lam_dst[nxt])[xr] = ab - s_m[k][lr];
        }
        term = wave_sum(term);
        if (lane == 0) rec[k] = term;
      }
      const double av = vr ? ab : -INFINITY;
      const double Mw = wave_max(av);
      const double Sw = wave_sum(av > -INFINITY ? exp(av - Mw) : 0.0);
      if (lane == 0) {
        rec[deg] = Mw;
        rec[deg + 1] = Sw;
      }
    }
    if (!SPARE) store_shifts(threadIdx.x, NT);
    return;
  }

  // more than kNodeDegLDS edges: wave 0 reads the messages from mfull (lane
  // group 0 holds every row of the tile)
  if (wv != 0) return;
#pragma unroll
  for (int r = 0; r < R; ++r) vx[r] = vx[r] && half == 0;
  double mux[R], a[R], qb[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    mux[r] = (vx[r] && fixed) ? nd.mu[x[r]] : 0.0;
    double asum = 0.0, qsum = 0.0;
    if (vx[r]) {
      for (int k = 0; k < deg; ++k) {
        const double m = mds[k].mfull[x[r]];
        asum += m;
        if (!fixed) qsum += exp(mds[k].lam_dst[cur][x[r]] - c_old + m);
      }
    }
    a[r] = vx[r] ? asum / deg : -INFINITY;
    qb[r] = qsum / deg;
  }
  // row x of the tile belongs to the 64-row record (x - row0) / 64: lane-row
  // r of a lane covers rows r * LPR + lrow, record (r * LPR) / RR
  for (int q = 0; q < TQ; ++q) {
    if (ti.row0 + q * RR >= n) break;
    double* __restrict__ rec = nd.tpart + (size_t)(ti.row0 / RR + q) * (deg + kRecExtra);
    for (int k = 0; k < deg; ++k) {
      double part = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!vx[r] || (r * LPR) / RR != q) continue;
        const double m = mds[k].mfull[x[r]];
        const double l = mds[k].lam_dst[cur][x[r]];
        double* __restrict__ Ln = mds[k].lam_dst[nxt];
        if (fixed) {
          if (mux[r] > 0.0) part += mux[r] * fabs(expm1(l + m));
          Ln[x[r]] = -m;
        } else {
          part += fabs(exp(l - c_old + m) - qb[r]);
          Ln[x[r]] = a[r] - m;
        }
      }
      part = wave_sum(part);
      if (lane == 0) rec[k] = part;
    }
    if (!fixed) {
      double am = -INFINITY;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if ((r * LPR) / RR == q) am = fmax(am, a[r]);
      const double Mw = wave_max(am);
      double sv = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if ((r * LPR) / RR == q) sv += (a[r] > -INFINITY) ? exp(a[r] - Mw) : 0.0;
      const double Sw = wave_sum(sv);
      if (lane == 0) {
        rec[deg] = Mw;
        rec[deg + 1] = Sw;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Separable messages on Cartesian grids (squared-Euclidean cost, D = 2).
// When every support of an instance is a row-major grid -- point p of node j
// at (R_j[p / B_j], C_j[p % B_j]), the last row possibly partial -- the cost
// splits, |x - y|^2 = (R_j[p] - R_k[u])^2 + (C_j[q] - C_k[v])^2, and so does
// the log-sum-exp of the message (eq. q), in two one-dimensional passes:
//   T(u, q) = log2 sum_v 2^(a(u, v) - kap (C_j[q] - C_k[v])^2)           (pass 0)
//   m(p, q) = ln2 log2 sum_u 2^(T(u, q) - kap (R_j[p] - R_k[u])^2) - c_k   (pass 1)
// with a = log2e (L_(k,j) + log gamma_k) over the source's points (absent
// points of a partial last row give -inf), kap = log2e / eps, and c_k the
// source's normaliser: n_k B_j + n_j A_k terms per message instead of n_j n_k.
//
// Both passes run one kernel over "lines" of a one-dimensional LSE
// convolution: out(o) = log2 sum_i 2^(s(i) - kap (z_o - y_i)^2).  With the
// square expanded, the y_i^2 part goes into the staged values s(i) and the
// z_o^2 part leaves the sum, so a term costs one FP64 FMA, s(i) + 2 kap z_o y_i,
// before its exponential:
//   pass 0: line u (source row), outputs q, inner v; s = a(u, v) - kap C_k[v]^2,
//           y = C_k[v], z = C_j[q]; stores Tt(q, u) = T(u, q) - kap R_k[u]^2;
//   pass 1: line q (destination column), outputs p, inner u; s = Tt(q, u),
//           y = R_k[u], z = R_j[p]; stores m(p B_j + q) in mfull.
// A block stages the values of its lines (every inner index, rows of odd
// stride so lanes on different lines hit different banks) and the inner
// coordinates in LDS, after loading each of its outputs' coordinate and
// shift into registers (up to kSepOut outputs per thread), so a block waits
// for memory once.
//
// Sums (FP32 core) follow the node kernel's contract: pairs of v_exp_f32
// terms of the FP64-reduced argument, added in FP32 and accumulated in FP64.
// From the third half-sweep of a call on, one pass shifted by the output's
// previous shift (the log2 of its largest pair sum, kept per output); an
// output whose sum leaves [2^kShiftLo, 2^kShiftHi] (terms may have overflowed
// or underflowed; a non-finite shift lands here too) is taken again in two
// passes (exact FP64 max, then the shifted sum).  The first two half-sweeps of
// a call take two passes; the FP64 variant (F64) always does, with FP64
// exponentials.
// ---------------------------------------------------------------------------
constexpr int kSepOut = 8;  // outputs per thread of a separable-pass block

template <bool F64, int PASS>
__global__ __launch_bounds__(64 * kSepWaves) void k_sep_pass(Tables tb) {
  extern __shared__ double s_dyn[];
  int bid = (int)blockIdx.x;
  if (PASS == 0) {
    if (bid < tb.n_fin) {
      // the finalise step of the previous launch's half-sweep, one block per instance
      __shared__ double sh_fin[kFinParts][2];
      fin_instance<kSepWaves>(tb, tb.fin_nodes, tb.fin_colour, tb.inst + bid, true, sh_fin);
      return;
    }
    bid -= tb.n_fin;
  }
  const SepItem it = (PASS == 0 ? tb.sep_items : tb.sep_items2)[bid];
  const CMsg& md = *(const CMsg*)(tb.msgs + it.msg);
  const InstState* st = tb.inst + it.inst;
  const long long t = st->vt[tb.colour];
  const long long t_first = st->t_first;
  if (st->vdone[tb.colour] != 0 || t < t_first || ((t & 1) == 1) != (tb.colour == 0)) return;
  const bool one = !F64 && t >= st->onepass_from;
  const int tid = threadIdx.x, lane = tid & 63;
  const int Ak = md.rows_src, Bk = md.cols_src, Aj = md.rows_dst, Bj = md.cols_dst;
  const int nk = md.n_src, nj = md.n_dst;
  const int outs = PASS == 0 ? Bj : Aj;   // outputs per line
  const int inner = PASS == 0 ? Bk : Ak;  // terms per output
  const int IS = (inner + 1) | 1;         // staged row stride (odd, > inner when inner is odd)
  const int IE = (inner + 1) & ~1;        // inner rounded up to even
  const int NL = it.nlines, NF = NL * outs;
  const double kap = kLog2e / md.eps;
  const int src_slot = (int)((t >> 1) % kSlots);
  const GDbl* __restrict__ lam = (const GDbl*)md.lam_src[src_slot];
  const GDbl* __restrict__ lg = (const GDbl*)md.lg_src;
  const GDbl* __restrict__ ys = (const GDbl*)md.supp_src;
  const GDbl* __restrict__ xs = (const GDbl*)md.supp_dst;
  GDblW* __restrict__ Tt = (GDblW*)md.sepT;
  GDblW* __restrict__ shift = PASS == 0 ? (GDblW*)md.sepM : (GDblW*)md.wmax;
  double* __restrict__ sy = s_dyn;       // [IE] inner coordinates
  double* __restrict__ sa = s_dyn + IE;  // [NL x IS] staged values
  // this thread's outputs f = tid + 256 i: coordinate z and previous shift
  // (clamped loads; f >= NF is never used)
  double zr[kSepOut], shr[kSepOut];
#pragma unroll
  for (int i = 0; i < kSepOut; ++i) {
    const int f = min(tid + 64 * kSepWaves * i, NF - 1);
    const int row = f / outs, o = f - row * outs, line = it.line0 + row;
    zr[i] = PASS == 0 ? xs[(size_t)o * 2 + 1] : xs[(size_t)min(o * Bj, nj - 1) * 2];
    const size_t si = PASS == 0 ? (size_t)line * Bj + o : (size_t)min(o * Bj + line, nj - 1);
    shr[i] = one ? shift[si] : 0.0;
  }
  // pass 1: the source's normaliser, from its tile records when its last
  // update (half-sweep t - 1) ran in this run, else its stored value
  double ck = 0.0;
  if (PASS == 1 && md.src_free) {
    if (t - 1 >= t_first) {
      const GDbl* __restrict__ srec = (const GDbl*)md.src_tpart;
      const int src_deg = md.src_deg, src_tiles = md.src_tiles;
      const int s_stride = src_deg + kRecExtra, s_tile = min(lane, src_tiles - 1);
      ck = tile_lse((const double*)srec, src_tiles, s_stride, src_deg, srec[(size_t)s_tile * s_stride + src_deg],
                    srec[(size_t)s_tile * s_stride + src_deg + 1]);
    } else {
      ck = *(const GDbl*)(md.c_src + src_slot);
    }
  }
  // stage: inner coordinates (pads 0), then the lines' values (pads -inf)
  for (int c = tid; c < IE; c += 64 * kSepWaves) {
    double y = 0.0;
    if (c < inner) y = PASS == 0 ? ys[(size_t)c * 2 + 1] : ys[(size_t)c * Bk * 2];
    sy[c] = y;
  }
  for (int idx = tid; idx < NL * inner; idx += 64 * kSepWaves) {
    const int l = idx / inner, c = idx - l * inner, line = it.line0 + l;
    double a;
    if (PASS == 0) {
      const int y = line * Bk + c;
      const int yc = y < nk ? y : nk - 1;
      const double cv = ys[(size_t)c * 2 + 1];
      const double av = lam[yc] + lg[yc];
      a = y < nk ? fma(-kap * cv, cv, kLog2e * av) : -INFINITY;
    } else {
      a = Tt[(size_t)line * Ak + c];
    }
    sa[l * IS + c] = a;
  }
  if (inner & 1)
    for (int l = tid; l < NL; l += 64 * kSepWaves) sa[l * IS + inner] = -INFINITY;
  __syncthreads();

#pragma unroll
  for (int i = 0; i < kSepOut; ++i) {
    const int f = tid + 64 * kSepWaves * i;
    if (f < NF) {
      const int row = f / outs, o = f - row * outs, line = it.line0 + row;
      const int x = o * Bj + line;  // pass 1: the output's point of node j
      const double z = zr[i], cf = 2.0 * kap * z;
      const double* __restrict__ ar = sa + row * IS;
      double base = shr[i], S = 0.0;
      float Mp = 0.0f;
      bool two = !one;
      if (one) {
#pragma unroll 4
        for (int c = 0; c < inner; c += 2) {
          const double d0 = fma(cf, sy[c], ar[c]) - base, d1 = fma(cf, sy[c + 1], ar[c + 1]) - base;
          const float p = exp2_hw((float)d0) + exp2_hw((float)d1);
          Mp = fmaxf(Mp, p);
          S += (double)p;
        }
        two = !(S >= kSumLo && S <= kSumHi);
      }
      if (two) {
        double M = -INFINITY;
#pragma unroll 4
        for (int c = 0; c < inner; ++c) M = fmax(M, fma(cf, sy[c], ar[c]));
        base = M;
        S = 0.0;
        Mp = 0.0f;
        if (M > -INFINITY) {
#pragma unroll 4
          for (int c = 0; c < inner; c += 2) {
            const double d0 = fma(cf, sy[c], ar[c]) - M, d1 = fma(cf, sy[c + 1], ar[c + 1]) - M;
            if (F64) {
              S += exp2(d0) + exp2(d1);
            } else {
              const float p = exp2_hw((float)d0) + exp2_hw((float)d1);
              Mp = fmaxf(Mp, p);
              S += (double)p;
            }
          }
        }
      }
      const double T = (base > -INFINITY && S > 0.0) ? base + log2(S) : -INFINITY;
      // next shift: the log2 of the largest pair sum (FP32 core), the exact max (F64)
      const double nsh = F64 ? base : (Mp > 0.0f ? base + log2((double)Mp) : -INFINITY);
      if (PASS == 0) {
        const double Ru = ys[(size_t)line * Bk * 2];
        Tt[(size_t)o * Ak + line] = T - kap * (z * z) - kap * (Ru * Ru);
        shift[(size_t)line * Bj + o] = nsh;
      } else if (x < nj) {
        ((GDblW*)md.mfull)[x] = T > -INFINITY ? kLn2 * (T - kap * (z * z)) - ck : -INFINITY;
        shift[x] = nsh;
      }
    }
  }
}

// Node stage of a separable instance, after its messages (the second pass
// wrote them to mfull): one wave per tile record (tb.rec_rows rows, lane =
// row; 64 / rec_rows records per 64-row tile, kSepWaves records per block),
// the stopping-sum terms of the state before the update, the update and the
// record, as k_node does.
__global__ __launch_bounds__(64 * kSepWaves) void k_node_sep(Tables tb, int n_tiles) {
  const int RR = tb.rec_rows, TQ = 64 / RR;
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int gw = (int)blockIdx.x * kSepWaves + wv;
  if (gw >= n_tiles * TQ) return;
  const TileItem ti = tb.tiles[gw / TQ];
  const int sub = gw - (gw / TQ) * TQ;
  const InstState* st = tb.inst + ti.inst;
  const long long t = st->vt[tb.colour];
  if (st->vdone[tb.colour] != 0 || t < st->t_first || ((t & 1) == 1) != (tb.colour == 0)) return;
  const int n = ti.n, deg = ti.deg;
  if (ti.row0 + sub * RR >= n) return;
  const NodeItem nd = tb.nodes[ti.node];
  const CMsg* __restrict__ mds = (const CMsg*)(tb.msgs + ti.msg0);
  const int cur = (int)(((t - 1) >> 1) % kSlots), nxt = (cur + 1) % kSlots;
  const int xr = ti.row0 + sub * RR + (lane < RR ? lane : 0);
  const bool vr = lane < RR && xr < n;
  const int xs = vr ? xr : ti.row0 + sub * RR;
  GDblW* __restrict__ rec = (GDblW*)(nd.tpart + (size_t)(ti.row0 / RR + sub) * (deg + kRecExtra));
  auto msg = [&](int k) -> double { return ((const GDbl*)mds[k].mfull)[xs]; };
  if (ti.fixed) {
    const double mu = vr ? ((const GDbl*)nd.mu)[xr] : 0.0;
    for (int k = 0; k < deg; ++k) {
      const double m = msg(k);
      double term = 0.0;
      if (vr) {
        const double l = ((const GDbl*)mds[k].lam_dst[cur])[xr];
        if (mu > 0.0) term = mu * fabs(expm1(l + m));
        ((GDblW*)mds[k].lam_dst[nxt])[xr] = -m;
      }
      term = wave_sum(term);
      if (lane == 0) rec[k] = term;
    }
  } else {
    const double c_old = *(const GDbl*)(nd.c + cur);
    double as = 0.0, qs = 0.0;
    for (int k = 0; k < deg; ++k) {
      const double m = msg(k);
      as += m;
      if (vr) qs += exp(((const GDbl*)mds[k].lam_dst[cur])[xr] - c_old + m);
    }
    const double ab = as / deg, qb = qs / deg;
    for (int k = 0; k < deg; ++k) {
      const double m = msg(k);
      double term = 0.0;
      if (vr) {
        term = fabs(exp(((const GDbl*)mds[k].lam_dst[cur])[xr] - c_old + m) - qb);
        ((GDblW*)mds[k].lam_dst[nxt])[xr] = ab - m;
      }
      term = wave_sum(term);
      if (lane == 0) rec[k] = term;
    }
    const double av = vr ? ab : -INFINITY;
    const double Mw = wave_max(av);
    const double Sw = wave_sum(av > -INFINITY ? exp(av - Mw) : 0.0);
    if (lane == 0) {
      rec[deg] = Mw;
      rec[deg + 1] = Sw;
    }
  }
}

// ---------------------------------------------------------------------------
// Messages whose source support is a uniform one-dimensional grid,
// y_j = y_0 + j h (j < n_src), for the squared-Euclidean cost.  One wave takes
// one message for 64 R destination rows x (any support; R rows per lane).
// With x_c the midpoint of the wave's smallest and largest row and
// kap = log2e / eps,
//   w(x, y_j) = C(j) + g(x) j + 2 kap (x - x_c) y_0 - kap x^2,
//   C(j) = log2e (L_(k,j) + log gamma_k)(y_j) - kap y_j^2 + 2 kap x_c y_j,
//   g(x) = 2 kap (x - x_c) h,
// so sum_j 2^w = 2^(theta + 2 kap (x - x_c) y_0 - kap x^2) * sum_j v_j rho^j
// with v_j = 2^(C(j) - theta), the same for the wave's rows, and rho = 2^g(x)
// per row: a polynomial in rho, summed by Horner's rule at one FP64 FMA per
// (row, column) pair.  Columns come 64 at a time from the last tile down
// (Horner in rho^64 across tiles).  Inside a tile every row of 16 lanes holds
// the tile's 64 values v (four registers), the lane's powers rho^0..rho^15
// stay in registers, and v_fmac_f64 with row_newbcast:q hands each lane
// column q of a 16-column group; the four groups combine in rho^16.
// theta is the largest C met so far, moved (and the partial sum rescaled) only
// when a column exceeds it by more than kGridSlack binades, so v <= 2^kGridSlack.
// The host takes this path only when 2 kap * (half the span of any 64 R rows)
// * |h| * max(n_src - 1, 64) <= kGridRange binades, so every power of rho
// formed here (up to rho^64) or summed (rho^j, j < n_src) stays within
// 2^(+-kGridRange): with v_j <= 2^kGridSlack in FP64 no term that matters
// underflows and no sum overflows.  Every step is FP64 (v and rho from exp2 in FP64), so the
// messages agree with the FP64 node kernel to rounding.  The update of each
// node follows in k_node_sep from the merged messages in mfull.
// ---------------------------------------------------------------------------
constexpr int kGridWaves = 4;          // waves (items) per block

// acc += a[lane q of acc's 16-lane row] * b (double-precision DPP row broadcast)
#define GMOT_FMAC_ROWBCAST(acc, a, b, Q) \
  asm("v_fmac_f64_dpp %0, %1, %2 row_newbcast:" #Q " row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(a), "v"(b))

// two rows per lane asks for four waves per SIMD (at most 128 VGPRs).
// EVAL: the FP64 evaluation pass -- every item regardless of its instance's
// loop state, the source's committed slot from tb.inst_slot and its stored
// normaliser, and the message written as column split 0 of the evaluation's
// partials (the other splits empty), as k_msg leaves them.  It also sums
// j v_j rho^j and j^2 v_j rho^j, so that the row's mean cost under the plan,
// sum_j B (x - y_j)^2 / sum_j B = d^2 - 2 d h S1 / S0 + h^2 S2 / S0 with
// d = x - y_0, goes to wmax[x] (the transport cost without a pair pass).
template <int R, bool EVAL>
__global__ __launch_bounds__(64 * kGridWaves, R == 2 ? 3 : 1) void k_msg_grid(Tables tb, int n_items) {
  __shared__ double s_v[kGridWaves][64];
  if (!EVAL && (int)blockIdx.x < tb.n_fin) {
    // the finalise step of the previous launch's half-sweep, one block per instance
    __shared__ double sh_fin[kFinParts][2];
    fin_instance<kGridWaves>(tb, tb.fin_nodes, tb.fin_colour, tb.inst + blockIdx.x, true, sh_fin);
    return;
  }
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int gw = ((int)blockIdx.x - tb.n_fin) * kGridWaves + wv;
  if (gw >= n_items) return;
  const TileItem ti = tb.tiles[gw];
  const InstState* st = tb.inst + ti.inst;
  long long t = 0;
  if (!EVAL) {
    t = st->vt[tb.colour];
    if (st->vdone[tb.colour] != 0 || t < st->t_first || ((t & 1) == 1) != (tb.colour == 0)) return;
  }
  const CMsg& md = *(const CMsg*)(tb.msgs + ti.msg0);
  const int n = md.n_dst, ns = md.n_src;
  const int src_slot = EVAL ? tb.inst_slot[2 * ti.inst + (1 - tb.colour)] : (int)((t >> 1) % kSlots);
  const GDbl* __restrict__ lam = (const GDbl*)md.lam_src[src_slot];
  const GDbl* __restrict__ lg = (const GDbl*)md.lg_src;
  const GDbl* __restrict__ ys = (const GDbl*)md.supp_src;
  const GDbl* __restrict__ xs = (const GDbl*)md.supp_dst;
  const double kap = kLog2e / md.eps;
  // this lane's rows row0 + 64 r + lane (clamped: rows past n compute a value
  // that is not stored); x_c the midpoint of the wave's rows
  int x[R];
  double xv[R], hi = -INFINITY, lo = -INFINITY;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    x[r] = ti.row0 + 64 * r + lane;
    xv[r] = xs[min(x[r], n - 1)];
    if (x[r] < n) {
      hi = fmax(hi, xv[r]);
      lo = fmax(lo, -xv[r]);
    }
  }
  const double xc = 0.5 * (wave_max(hi) - wave_max(lo));
  const double y0 = ys[0];
  const double h = ns > 1 ? (ys[ns - 1] - y0) / (double)(ns - 1) : 0.0;
  double dx[R], pw[R][16], r16[R], r64[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    dx[r] = xv[r] - xc;
    const double rho = exp2(2.0 * kap * dx[r] * h);
    pw[r][0] = 1.0;
#pragma unroll
    for (int q = 1; q < 16; ++q) pw[r][q] = pw[r][q - 1] * rho;
    r16[r] = pw[r][15] * rho;
    r64[r] = (r16[r] * r16[r]) * (r16[r] * r16[r]);
  }
  const double cxc = 2.0 * kap * xc;
  // column data of tile J (lane = column 64 J + lane, clamped; past n_src: no term)
  auto c_of = [&](double l, double g, double y, bool ok) -> double {
    return ok ? fma(cxc - kap * y, y, kLog2e * (l + g)) : -INFINITY;
  };
  const int nt = (ns + 63) / 64;
  // columns two tiles ahead: tile J's in (l_n, g_n, y_n), tile J - 1's in
  // (l_m, g_m, y_m), loaded while tile J + 1 is summed (clamped indexes)
  int jn = min((nt - 1) * 64 + lane, ns - 1);
  double l_n = lam[jn], g_n = lg[jn], y_n = ys[jn];
  jn = max(nt - 2, 0) * 64 + lane;
  double l_m = lam[jn], g_m = lg[jn], y_m = ys[jn];
  double theta = -INFINITY, P[R], P1[EVAL ? R : 1], P2[EVAL ? R : 1];
#pragma unroll
  for (int r = 0; r < R; ++r) P[r] = 0.0;
#pragma unroll
  for (int r = 0; r < (EVAL ? R : 1); ++r) P1[r] = P2[r] = 0.0;
  double* __restrict__ sv = s_v[wv];
  for (int J = nt - 1; J >= 0; --J) {
    const double C = c_of(l_n, g_n, y_n, J * 64 + lane < ns);
    l_n = l_m;
    g_n = g_m;
    y_n = y_m;
    if (J > 1) {
      jn = (J - 2) * 64 + lane;
      l_m = lam[jn];
      g_m = lg[jn];
      y_m = ys[jn];
    }
    if (__any(C > theta + kGridSlack)) {
      const double m = wave_max(C);
      if (theta > -INFINITY) {
        const double f = exp2(theta - m);
#pragma unroll
        for (int r = 0; r < R; ++r) P[r] *= f;
        if (EVAL)
#pragma unroll
          for (int r = 0; r < R; ++r) {
            P1[r] *= f;
            P2[r] *= f;
          }
      }
      theta = m;
    }
    sv[lane] = C > -INFINITY ? exp2(C - theta) : 0.0;
    wave_sync();
    double vc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) vc[c] = sv[16 * c + (lane & 15)];
    wave_sync();
    double S[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) S[r][c] = 0.0;
    // the four groups (and the rows) interleaved: 4 R independent chains
#define GMOT_GRID_COL(Q)                                              \
  _Pragma("unroll") for (int r = 0; r < R; ++r) {                     \
    GMOT_FMAC_ROWBCAST(S[r][0], vc[0], pw[r][Q], Q);                  \
    GMOT_FMAC_ROWBCAST(S[r][1], vc[1], pw[r][Q], Q);                  \
    GMOT_FMAC_ROWBCAST(S[r][2], vc[2], pw[r][Q], Q);                  \
    GMOT_FMAC_ROWBCAST(S[r][3], vc[3], pw[r][Q], Q);                  \
  }
    GMOT_GRID_COL(0) GMOT_GRID_COL(1) GMOT_GRID_COL(2) GMOT_GRID_COL(3)
    GMOT_GRID_COL(4) GMOT_GRID_COL(5) GMOT_GRID_COL(6) GMOT_GRID_COL(7)
    GMOT_GRID_COL(8) GMOT_GRID_COL(9) GMOT_GRID_COL(10) GMOT_GRID_COL(11)
    GMOT_GRID_COL(12) GMOT_GRID_COL(13) GMOT_GRID_COL(14) GMOT_GRID_COL(15)
#undef GMOT_GRID_COL
#pragma unroll
    for (int r = 0; r < R; ++r)
      P[r] = fma(P[r], r64[r], fma(fma(fma(S[r][3], r16[r], S[r][2]), r16[r], S[r][1]), r16[r], S[r][0]));
    if (EVAL) {
      // the same sums with the coefficients j v_j and j^2 v_j (j the column)
      double w1[4], w2[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double jj = (double)(J * 64 + 16 * c + (lane & 15));
        w1[c] = jj * vc[c];
        w2[c] = jj * w1[c];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double T1[4] = {0.0, 0.0, 0.0, 0.0}, T2[4] = {0.0, 0.0, 0.0, 0.0};
#define GMOT_GRID_MOM(Q)                                    \
  GMOT_FMAC_ROWBCAST(T1[0], w1[0], pw[r][Q], Q);            \
  GMOT_FMAC_ROWBCAST(T1[1], w1[1], pw[r][Q], Q);            \
  GMOT_FMAC_ROWBCAST(T1[2], w1[2], pw[r][Q], Q);            \
  GMOT_FMAC_ROWBCAST(T1[3], w1[3], pw[r][Q], Q);            \
  GMOT_FMAC_ROWBCAST(T2[0], w2[0], pw[r][Q], Q);            \
  GMOT_FMAC_ROWBCAST(T2[1], w2[1], pw[r][Q], Q);            \
  GMOT_FMAC_ROWBCAST(T2[2], w2[2], pw[r][Q], Q);            \
  GMOT_FMAC_ROWBCAST(T2[3], w2[3], pw[r][Q], Q);
        GMOT_GRID_MOM(0) GMOT_GRID_MOM(1) GMOT_GRID_MOM(2) GMOT_GRID_MOM(3)
        GMOT_GRID_MOM(4) GMOT_GRID_MOM(5) GMOT_GRID_MOM(6) GMOT_GRID_MOM(7)
        GMOT_GRID_MOM(8) GMOT_GRID_MOM(9) GMOT_GRID_MOM(10) GMOT_GRID_MOM(11)
        GMOT_GRID_MOM(12) GMOT_GRID_MOM(13) GMOT_GRID_MOM(14) GMOT_GRID_MOM(15)
#undef GMOT_GRID_MOM
        P1[r] = fma(P1[r], r64[r], fma(fma(fma(T1[3], r16[r], T1[2]), r16[r], T1[1]), r16[r], T1[0]));
        P2[r] = fma(P2[r], r64[r], fma(fma(fma(T2[3], r16[r], T2[2]), r16[r], T2[1]), r16[r], T2[0]));
      }
    }
  }
  // the source's normaliser c_k, from its tile records when its last update
  // (half-sweep t - 1) ran in this run, else (and in the evaluation) its
  // stored value
  double ck = 0.0;
  if (md.src_free) {
    if (!EVAL && t - 1 >= st->t_first) {
      const GDbl* __restrict__ srec = (const GDbl*)md.src_tpart;
      const int src_deg = md.src_deg, src_tiles = md.src_tiles;
      const int s_stride = src_deg + kRecExtra, s_tile = min(lane, src_tiles - 1);
      ck = tile_lse((const double*)srec, src_tiles, s_stride, src_deg, srec[(size_t)s_tile * s_stride + src_deg],
                    srec[(size_t)s_tile * s_stride + src_deg + 1]);
    } else {
      ck = *(const GDbl*)(md.c_src + src_slot);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (x[r] < n) {
      const double e = theta + fma(2.0 * kap * dx[r], y0, -kap * xv[r] * xv[r]);
      const bool fin = theta > -INFINITY && P[r] > 0.0;
      if (EVAL) {
        // log2 of the sum without the -|x|^2 / eps the merge subtracts, c_k included
        const double l2 = fin ? e + log2(P[r]) + kap * xv[r] * xv[r] - kLog2e * ck : -INFINITY;
        double2* __restrict__ part = md.partial + (size_t)x[r] * md.ns;
        part[0] = make_double2(l2, fin ? 1.0 : 0.0);
        for (int sp = 1; sp < md.ns; ++sp) part[sp] = make_double2(-INFINITY, 0.0);
        const double d = xv[r] - y0;
        md.wmax[x[r]] = fin ? fma(d, d, h * fma(-2.0 * d, P1[r] / P[r], h * (P2[r] / P[r]))) : 0.0;
      } else {
        ((GDblW*)md.mfull)[x[r]] = fin ? kLn2 * (e + log2(P[r])) - ck : -INFINITY;
      }
    }
}
#undef GMOT_FMAC_ROWBCAST

// ---------------------------------------------------------------------------
// Separable passes on uniform grids by Horner's rule (FP64).  Each pass of a
// separable message (the two one-dimensional LSE convolutions above) is, per
// line, a one-dimensional message from uniformly spaced inputs y_i = y_0 + i h
// to the line's outputs z_o:
//   out(o) = log2 sum_i 2^(s(i) + 2 kap z_o y_i),   s(i) = staged value - kap y_i^2,
// summed as in k_msg_grid: with z_c the midpoint of the wave's outputs,
//   out(o) = theta + log2 sum_i v_i rho_o^i + 2 kap (z_o - z_c) y_0,
//   v_i = 2^(C(i) - theta),  C(i) = s(i) + 2 kap z_c y_i,  rho_o = 2^(2 kap (z_o - z_c) h).
// One wave takes one task: 64 outputs (lane = output) of kSepLines lines of
// one message; the powers of each lane's rho are formed once, and for each
// line the lanes compute the line's values v (lane = input, 64 per tile),
// exchange them through LDS so that every 16-lane row holds all of them, and
// sum with the row broadcast of v_fmac_f64, only over the 16-input groups
// the inputs fill.  The host takes this path only when every grid coordinate
// list is uniform and, per pass, 2 kap * (half the span of 64 consecutive
// outputs) * |h| * W <= kGridRange, with W the largest power of rho formed:
// 16 g - 1 for g = ceil(inner / 16) <= 4 groups in one tile, max(inner - 1, 64)
// over several tiles.  Pass 0 stores Tt(q, u) = T(u, q) - kap C_j[q]^2 -
// kap R_k[u]^2, pass 1 the message in mfull, as k_sep_pass does.
// ---------------------------------------------------------------------------
constexpr int kSepLines = kSepTaskLines;  // lines per task of a separable Horner pass

#define GMOT_FMAC_ROWBCAST_S(acc, a, b, Q) \
  asm("v_fmac_f64_dpp %0, %1, %2 row_newbcast:" #Q " row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(a), "v"(b))

// sum over the NG groups of 16 inputs of one tile: sum_c rho^(16 c) sum_q v[16 c + q] rho^q
template <int NG>
__device__ inline double horner_tile(const double* vc, const double* pw, double r16) {
  double S[4] = {0.0, 0.0, 0.0, 0.0};
#define GMOT_SEP_COL(Q)                                                  \
  GMOT_FMAC_ROWBCAST_S(S[0], vc[0], pw[Q], Q);                           \
  if (NG > 1) GMOT_FMAC_ROWBCAST_S(S[1], vc[1], pw[Q], Q);               \
  if (NG > 2) GMOT_FMAC_ROWBCAST_S(S[2], vc[2], pw[Q], Q);               \
  if (NG > 3) GMOT_FMAC_ROWBCAST_S(S[3], vc[3], pw[Q], Q);
  GMOT_SEP_COL(0) GMOT_SEP_COL(1) GMOT_SEP_COL(2) GMOT_SEP_COL(3)
  GMOT_SEP_COL(4) GMOT_SEP_COL(5) GMOT_SEP_COL(6) GMOT_SEP_COL(7)
  GMOT_SEP_COL(8) GMOT_SEP_COL(9) GMOT_SEP_COL(10) GMOT_SEP_COL(11)
  GMOT_SEP_COL(12) GMOT_SEP_COL(13) GMOT_SEP_COL(14) GMOT_SEP_COL(15)
#undef GMOT_SEP_COL
  if (NG == 1) return S[0];
  if (NG == 2) return fma(S[1], r16, S[0]);
  if (NG == 3) return fma(fma(S[2], r16, S[1]), r16, S[0]);
  return fma(fma(fma(S[3], r16, S[2]), r16, S[1]), r16, S[0]);
}

// EVAL: the FP64 evaluation pass (as for k_msg_grid): every task, the
// source's committed slot and stored normaliser, the message as split 0 of
// the evaluation's partials.  It also leaves the mean cost of each plan row:
// with the cost |x - y|^2 = (R_j - R_k)^2 + (C_j - C_k)^2, pass 0 sums the
// moments i v_i rho^i and i^2 v_i rho^i of its line and stores the line's mean
// of (C_j[q] - C_k[i])^2 (d^2 - 2 d h S1 / S0 + h^2 S2 / S0, d = C_j[q] - C_k[0])
// in sepM at Tt's index; pass 1 weights the inputs by the same moments of
// (R_j[p] - R_k[u])^2 and by that stored mean, and writes the row's mean
// cost sum_y B C / sum_y B to wmax[x] (the transport cost without a pair pass).
template <int PASS, bool EVAL>
__global__ __launch_bounds__(64 * kSepWaves) void k_sep_horner(Tables tb, int n_tasks) {
  __shared__ double s_v[kSepWaves][64];
  __shared__ double s_m[EVAL && PASS == 1 ? kSepWaves : 1][64];
  int bid = (int)blockIdx.x;
  if (PASS == 0 && !EVAL) {
    if (bid < tb.n_fin) {
      // the finalise step of the previous launch's half-sweep, one block per instance
      __shared__ double sh_fin[kFinParts][2];
      fin_instance<kSepWaves>(tb, tb.fin_nodes, tb.fin_colour, tb.inst + bid, true, sh_fin);
      return;
    }
    bid -= tb.n_fin;
  }
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int w = bid * kSepWaves + wv;
  if (w >= n_tasks) return;
  const SepTask tk = (PASS == 0 ? tb.sep_tasks : tb.sep_tasks2)[w];
  const InstState* st = tb.inst + tk.inst;
  long long t = 0;
  if (!EVAL) {
    t = st->vt[tb.colour];
    if (st->vdone[tb.colour] != 0 || t < st->t_first || ((t & 1) == 1) != (tb.colour == 0)) return;
  }
  const CMsg& md = *(const CMsg*)(tb.msgs + tk.msg);
  const int Ak = md.rows_src, Bk = md.cols_src, Bj = md.cols_dst, Aj = md.rows_dst;
  const int nk = md.n_src, nj = md.n_dst;
  const int outs = PASS == 0 ? Bj : Aj;     // outputs per line
  const int inner = PASS == 0 ? Bk : Ak;    // inputs per output
  const int lines = PASS == 0 ? Ak : Bj;
  const int src_slot = EVAL ? tb.inst_slot[2 * tk.inst + (1 - tb.colour)] : (int)((t >> 1) % kSlots);
  const GDbl* __restrict__ lam = (const GDbl*)md.lam_src[src_slot];
  const GDbl* __restrict__ lg = (const GDbl*)md.lg_src;
  const GDbl* __restrict__ ys = (const GDbl*)md.supp_src;
  const GDbl* __restrict__ xs = (const GDbl*)md.supp_dst;
  const GDbl* __restrict__ Tr = (const GDbl*)md.sepT;
  const double kap = kLog2e / md.eps;
  const int o = tk.o0 + lane;
  const bool ov = o < outs;
  const int oc = min(o, outs - 1);
  // input coordinate i of the pass and the output coordinate of this lane
  auto yin = [&](int i) -> double { return PASS == 0 ? ys[(size_t)i * 2 + 1] : ys[(size_t)i * Bk * 2]; };
  const double z = PASS == 0 ? xs[(size_t)oc * 2 + 1] : xs[(size_t)oc * Bj * 2];
  const double zc = 0.5 * (wave_max(ov ? z : -INFINITY) - wave_max(ov ? -z : -INFINITY));
  const double y0 = yin(0);
  const double h = inner > 1 ? (yin(inner - 1) - y0) / (double)(inner - 1) : 0.0;
  const double dz = z - zc;
  const double rho = exp2(2.0 * kap * dz * h);
  double pw[16];
  pw[0] = 1.0;
#pragma unroll
  for (int q = 1; q < 16; ++q) pw[q] = pw[q - 1] * rho;
  const double r16 = pw[15] * rho;
  const double czc = 2.0 * kap * zc;
  const int nt = (inner + 63) / 64;
  const int ng = nt > 1 ? 4 : (inner + 15) / 16;  // 16-input groups of a tile
  // pass 1: the source's normaliser c_k (its stored value in the evaluation)
  double ck = 0.0;
  if (PASS == 1 && md.src_free) {
    if (!EVAL && t - 1 >= st->t_first) {
      const GDbl* __restrict__ srec = (const GDbl*)md.src_tpart;
      const int src_deg = md.src_deg, src_tiles = md.src_tiles;
      const int s_stride = src_deg + kRecExtra, s_tile = min(lane, src_tiles - 1);
      ck = tile_lse((const double*)srec, src_tiles, s_stride, src_deg, srec[(size_t)s_tile * s_stride + src_deg],
                    srec[(size_t)s_tile * s_stride + src_deg + 1]);
    } else {
      ck = *(const GDbl*)(md.c_src + src_slot);
    }
  }
  double* __restrict__ sv = s_v[wv];
  const int l_end = min(tk.line + kSepLines, lines);
  // a line's inputs of its first-summed tile (the last): the coordinate is the
  // same for every line, the values of the next line are loaded while the
  // current one is summed (clamped indexes)
  const int i_top = (nt - 1) * 64 + lane, ic_top = min(i_top, inner - 1);
  const double y_top = yin(ic_top);
  double ra, rb;  // raw inputs of (line, top tile): pass 0 L and log gamma, pass 1 Tt
  auto load_top = [&](int line, double& a, double& b) {
    if (PASS == 0) {
      const int idx = min(line * Bk + ic_top, nk - 1);
      a = lam[idx];
      b = lg[idx];
    } else {
      a = Tr[(size_t)line * Ak + ic_top];
      b = 0.0;
    }
  };
  load_top(tk.line, ra, rb);
  for (int line = tk.line; line < l_end; ++line) {
    double theta = -INFINITY, P = 0.0, P1 = 0.0, P2 = 0.0, P3 = 0.0;
    const double ra_c = ra, rb_c = rb;
    if (line + 1 < l_end) load_top(line + 1, ra, rb);
    for (int J = nt - 1; J >= 0; --J) {
      const int i = J * 64 + lane;
      const int ic = min(i, inner - 1);
      const double y = J == nt - 1 ? y_top : yin(ic);
      double s;
      if (PASS == 0) {
        double l, g;
        if (J == nt - 1) {
          l = ra_c;
          g = rb_c;
        } else {
          const int idx = min(line * Bk + ic, nk - 1);
          l = lam[idx];
          g = lg[idx];
        }
        s = (i < inner && line * Bk + i < nk) ? fma(-kap * y, y, kLog2e * (l + g)) : -INFINITY;
      } else {
        const double tv = J == nt - 1 ? ra_c : Tr[(size_t)line * Ak + ic];
        s = i < inner ? tv : -INFINITY;
      }
      const double C = s > -INFINITY ? fma(czc, y, s) : -INFINITY;
      // a line's first tile starts from the first input's value (any value
      // within the slack below the maximum serves; v_i <= 2^kGridSlack)
      if (J == nt - 1) theta = lane_read(C, 0);
      if (__any(C > theta + kGridSlack)) {
        const double m = wave_max(C);
        if (J != nt - 1 && theta > -INFINITY) {
          const double f = exp2(theta - m);
          P *= f;
          if (EVAL) {
            P1 *= f;
            P2 *= f;
            P3 *= f;
          }
        }
        theta = m;
      }
      const double vl = C > -INFINITY ? exp2(C - theta) : 0.0;
      sv[lane] = vl;
      // pass 1: the input's stored mean of the first pass's squared distance
      if (EVAL && PASS == 1) s_m[wv][lane] = vl * ((const GDbl*)md.sepM)[(size_t)line * Ak + ic];
      wave_sync();
      double vc[4], w1[4], w2[4], w3[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        vc[c] = sv[16 * c + (lane & 15)];
        if (EVAL) {
          const double jj = (double)(J * 64 + 16 * c + (lane & 15));
          w1[c] = jj * vc[c];
          w2[c] = jj * w1[c];
          w3[c] = PASS == 1 ? s_m[wv][16 * c + (lane & 15)] : 0.0;
        }
      }
      wave_sync();
      double St, St1 = 0.0, St2 = 0.0, St3 = 0.0;
      switch (ng) {
        case 1:
          St = horner_tile<1>(vc, pw, r16);
          if (EVAL) {
            St1 = horner_tile<1>(w1, pw, r16);
            St2 = horner_tile<1>(w2, pw, r16);
            if (PASS == 1) St3 = horner_tile<1>(w3, pw, r16);
          }
          break;
        case 2:
          St = horner_tile<2>(vc, pw, r16);
          if (EVAL) {
            St1 = horner_tile<2>(w1, pw, r16);
            St2 = horner_tile<2>(w2, pw, r16);
            if (PASS == 1) St3 = horner_tile<2>(w3, pw, r16);
          }
          break;
        case 3:
          St = horner_tile<3>(vc, pw, r16);
          if (EVAL) {
            St1 = horner_tile<3>(w1, pw, r16);
            St2 = horner_tile<3>(w2, pw, r16);
            if (PASS == 1) St3 = horner_tile<3>(w3, pw, r16);
          }
          break;
        default:
          St = horner_tile<4>(vc, pw, r16);
          if (EVAL) {
            St1 = horner_tile<4>(w1, pw, r16);
            St2 = horner_tile<4>(w2, pw, r16);
            if (PASS == 1) St3 = horner_tile<4>(w3, pw, r16);
          }
          break;
      }
      if (J == nt - 1) {
        P = St;
        P1 = St1;
        P2 = St2;
        P3 = St3;
      } else {
        const double r64 = (r16 * r16) * (r16 * r16);
        P = fma(P, r64, St);
        if (EVAL) {
          P1 = fma(P1, r64, St1);
          P2 = fma(P2, r64, St2);
          P3 = fma(P3, r64, St3);
        }
      }
    }
    // EVAL: the line's mean of the pass's squared distance (z - y_i)^2 under
    // the weights v_i rho^i, plus (pass 1) the inputs' stored first-pass means
    double mc = 0.0;
    if (EVAL && theta > -INFINITY && P > 0.0) {
      const double d = z - y0;
      mc = fma(d, d, h * fma(-2.0 * d, P1 / P, h * (P2 / P)));
      if (PASS == 1) mc += P3 / P;
    }
    const double T = (theta > -INFINITY && P > 0.0) ? theta + log2(P) + 2.0 * kap * dz * y0 : -INFINITY;
    if (PASS == 0) {
      if (ov) {
        const double Ru = ys[(size_t)line * Bk * 2];
        ((GDblW*)md.sepT)[(size_t)o * Ak + line] = T - kap * (z * z) - kap * (Ru * Ru);
        if (EVAL) md.sepM[(size_t)o * Ak + line] = mc;
      }
    } else {
      const int x = o * Bj + line;
      if (ov && x < nj) {
        if (EVAL) {
          // log2 of the sum without the -|x|^2 / eps the merge subtracts
          // (here the -kap C_j[q]^2 of the first pass is |x|^2's second part)
          const double l2 = T > -INFINITY ? T - kap * (z * z) + kap * (xs[(size_t)x * 2] * xs[(size_t)x * 2] +
                                                                      xs[(size_t)x * 2 + 1] * xs[(size_t)x * 2 + 1]) -
                                                kLog2e * ck
                                          : -INFINITY;
          double2* __restrict__ part = md.partial + (size_t)x * md.ns;
          part[0] = make_double2(l2, T > -INFINITY ? 1.0 : 0.0);
          for (int sp = 1; sp < md.ns; ++sp) part[sp] = make_double2(-INFINITY, 0.0);
          md.wmax[x] = mc;
        } else {
          ((GDblW*)md.mfull)[x] = T > -INFINITY ? kLn2 * (T - kap * (z * z)) - ck : -INFINITY;
        }
      }
    }
  }
}
#undef GMOT_FMAC_ROWBCAST_S

// ---------------------------------------------------------------------------
// Finalise kernel: one block of kFinWaves waves per instance, one wave per
// node of the class (nodes w, w + kFinWaves, ...): per-edge terms summed over
// the node's tile records (lanes over tiles), and for free nodes
// c_j = LSE over the tile records of abar; then the block sums the terms in a
// fixed order and thread 0 takes the stop decision.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64 * kFinWaves) void k_finalize(Tables tb) {
  __shared__ double sh[kFinParts][2];
  fin_instance<kFinWaves>(tb, tb.nodes, tb.colour, tb.inst + blockIdx.x, false, sh);
}

// ---------------------------------------------------------------------------
// Node-sequential (Gauss-Seidel) update of one node (one block), after k_msg
// wrote the column-split partials of every message into node j from its
// neighbours' current potentials: merge them (m_{k->j}) and write the node's
// new potentials into `slot` in the closed form of Theorem tree_dual_var
// (Prop. equi): constrained L_(j,k) = -m_{k->j}; free L_(j,k) = abar -
// m_{k->j}, abar = mean_k m_{k->j}, with the normaliser c_j = LSE_x abar
// (the potential being L - c_j), in FP64.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_gs_update(Tables tb, int node_item, int slot) {
  __shared__ double sh[4];
  const NodeItem nd = tb.nodes[node_item];
  const int n = nd.n, deg = nd.deg;
  const MsgDesc* __restrict__ mds = tb.msgs + nd.msg0;
  const int dim = mds[0].dim;
  const bool sq = mds[0].cost_kind == 0;
  const double* __restrict__ xs = mds[0].supp_dst;
  double mx = -INFINITY;
  for (int x = threadIdx.x; x < n; x += kBlock) {
    const double x2 = sq ? sq_norm(xs, dim, x) : 0.0;
    double as = 0.0;
    for (int k = 0; k < deg; ++k) {
      const double m = merge_row(mds[k], x, x2);
      mds[k].mfull[x] = m;
      as += m;
    }
    const double ab = nd.fixed ? 0.0 : as / deg;
    for (int k = 0; k < deg; ++k) mds[k].lam_dst[slot][x] = (nd.fixed ? 0.0 : ab) - mds[k].mfull[x];
    if (!nd.fixed) {
      nd.abar[x] = ab;
      mx = fmax(mx, ab);
    }
  }
  if (nd.fixed) return;
  const double M = block_max(mx, sh);
  double sum = 0.0;
  if (M > -INFINITY)
    for (int x = threadIdx.x; x < n; x += kBlock) sum += exp(nd.abar[x] - M);
  const double S = block_sum(sum, sh);
  if (threadIdx.x == 0) nd.c[slot] = (M > -INFINITY && S > 0.0) ? M + log(S) : -INFINITY;
}

// ---------------------------------------------------------------------------
// Evaluation node pass (one block per node, given slot): merge the splits,
// stopping-sum terms of the state, qbar (the node marginal q_bar_j), and
// <Lam, mu> (constrained) or rho_j and its spread in x (free).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_node_eval(Tables tb, int slot) {
  __shared__ double sh[4];
  const NodeItem nd = tb.nodes[blockIdx.x];
  if (slot < 0) slot = tb.inst_slot[2 * nd.inst + tb.colour];
  const int n = nd.n, deg = nd.deg;
  const MsgDesc* __restrict__ mds = tb.msgs + nd.msg0;
  const int dim = mds[0].dim;
  const bool sq = mds[0].cost_kind == 0;
  const double* __restrict__ xs = mds[0].supp_dst;
  const double cj = nd.c ? nd.c[slot] : 0.0;

  for (int x = threadIdx.x; x < n; x += kBlock) {
    const double x2 = sq ? sq_norm(xs, dim, x) : 0.0;
    const double lgx = nd.lg[x];
    double qsum = 0.0;
    for (int k = 0; k < deg; ++k) {
      const MsgDesc& md = mds[k];
      const double m = merge_row(md, x, x2);
      md.mfull[x] = m;
      qsum += exp(md.lam_dst[slot][x] - cj + lgx + m);
    }
    nd.qbar[x] = qsum / deg;
  }
  __syncthreads();
  double e_sum = 0.0, e_max = 0.0;
  for (int k = 0; k < deg; ++k) {
    const MsgDesc& md = mds[k];
    double part = 0.0, sq = 0.0, sl = 0.0, sc = 0.0;
    for (int x = threadIdx.x; x < n; x += kBlock) {
      const double l = md.lam_dst[slot][x] - cj;
      const double q = exp(l + nd.lg[x] + md.mfull[x]);
      const double ref = nd.fixed ? nd.mu[x] : nd.qbar[x];
      part += fabs(q - ref);
      // the plan's marginal on this node and its sums for the objective
      if (q > 0.0) {
        sq += q;
        sl += q * l;
        if (md.grid) sc += q * md.wmax[x];
      }
    }
    const double tot = block_sum(part, sh);
    e_sum += tot;
    e_max = fmax(e_max, tot);
    sq = block_sum(sq, sh);
    sl = block_sum(sl, sh);
    sc = block_sum(sc, sh);
    if (threadIdx.x == 0) tb.msg_eval[nd.msg0 + k] = make_double4(sq, sl, sc, 0.0);
  }
  double v0 = 0.0, lo = INFINITY, hi = -INFINITY;
  if (nd.fixed) {
    for (int k = 0; k < deg; ++k) {
      const double* Ls = mds[k].lam_dst[slot];
      for (int x = threadIdx.x; x < n; x += kBlock) {
        const double l = Ls[x];
        if (nd.mu[x] > 0.0 && isfinite(l)) v0 += l * nd.mu[x];
      }
    }
    v0 = block_sum(v0, sh);
    lo = hi = 0.0;
  } else {
    for (int x = threadIdx.x; x < n; x += kBlock) {
      double tot = 0.0;
      for (int k = 0; k < deg; ++k) tot += mds[k].lam_dst[slot][x] - cj;
      v0 += tot;
      lo = fmin(lo, tot);
      hi = fmax(hi, tot);
    }
    v0 = block_sum(v0, sh) / n;
    lo = -block_max(-lo, sh);
    hi = block_max(hi, sh);
  }
  if (threadIdx.x == 0) tb.node_eval[nd.err_idx] = make_double4(e_sum, e_max, v0, hi - lo);
}

__global__ void k_stamp(InstState* inst, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) inst[i].clk_start = wall_clock64();
}

// one block per segment: zero its doubles (vector stores)
__global__ __launch_bounds__(kBlock) void k_zero_segs(const ZeroSeg* segs) {
  const ZeroSeg sg = segs[blockIdx.x];
  for (int64_t i = threadIdx.x; i < sg.len; i += kBlock) sg.dst[i] = 0.0;
}

// ---------------------------------------------------------------------------
// FP64 pair pass: for each plan, sum_xy C B, sum_xy B (log B - log M - 1)
// and sum_xy B over a (256 rows x ncols) tile.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_pairs(const EdgeDesc* edges, const PairItem* items, double4* out) {
  __shared__ double sh[4];
  __shared__ double s_b[kChunk];
  __shared__ double s_y[kChunk * 3];
  __shared__ double s_g[kChunk];
  const PairItem it = items[blockIdx.x];
  const EdgeDesc ed = edges[it.edge];
  const int x = it.row0 + threadIdx.x;
  const bool vx = x < ed.n_a;
  const bool sq = ed.cost_kind == 0;
  const double ca = ed.c_a ? *ed.c_a : 0.0;
  const double cb = ed.c_b ? *ed.c_b : 0.0;
  const double inv_eps = 1.0 / ed.eps;
  double ax = -INFINITY, lax = 0.0, xp[3] = {0.0, 0.0, 0.0};
  if (vx) {
    lax = ed.lam_a[x] - ca;
    ax = lax + ed.lg_a[x];
    if (sq)
      for (int d = 0; d < ed.dim; ++d) xp[d] = ed.supp_a[(size_t)x * ed.dim + d];
  }
  double sT = 0.0, sH = 0.0, sM = 0.0;
  for (int c0 = 0; c0 < it.ncols; c0 += kChunk) {
    const int cn = min(kChunk, it.ncols - c0);
    __syncthreads();
    if (threadIdx.x < cn) {
      const int y = it.col0 + c0 + threadIdx.x;
      s_b[threadIdx.x] = ed.lam_b[y] - cb;
      s_g[threadIdx.x] = ed.lg_b[y];
      if (sq)
        for (int d = 0; d < ed.dim; ++d) s_y[threadIdx.x * 3 + d] = ed.supp_b[(size_t)y * ed.dim + d];
    }
    __syncthreads();
    if (vx) {
      for (int c = 0; c < cn; ++c) {
        const int y = it.col0 + c0 + c;
        double C;
        if (sq) {
          C = 0.0;
          for (int d = 0; d < ed.dim; ++d) {
            const double df = xp[d] - s_y[c * 3 + d];
            C = fma(df, df, C);
          }
        } else {
          C = (double)ed.cost[(size_t)x * ed.n_b + y];
        }
        const double lb = s_b[c];
        const double ce = C * inv_eps;
        const double B = exp(ax + lb + s_g[c] - ce);
        if (B > 0.0) {
          sT += C * B;
          sH += B * (lax + lb - ce - 1.0);
          sM += B;
        }
      }
    }
  }
  sT = block_sum(sT, sh);
  sH = block_sum(sH, sh);
  sM = block_sum(sM, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = make_double4(sT, sH, sM, (double)it.edge);
}

__global__ __launch_bounds__(kBlock) void k_coupling(const EdgeDesc* edp, double* out) {
  const EdgeDesc ed = *edp;
  const double ca = ed.c_a ? *ed.c_a : 0.0;
  const double cb = ed.c_b ? *ed.c_b : 0.0;
  const size_t total = (size_t)ed.n_a * ed.n_b;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (size_t)gridDim.x * kBlock) {
    const int x = (int)(i / ed.n_b), y = (int)(i % ed.n_b);
    double C;
    if (ed.cost_kind == 0) {
      C = 0.0;
      for (int d = 0; d < ed.dim; ++d) {
        const double df = ed.supp_a[(size_t)x * ed.dim + d] - ed.supp_b[(size_t)y * ed.dim + d];
        C = fma(df, df, C);
      }
    } else {
      C = (double)ed.cost[i];
    }
    out[i] = exp((ed.lam_a[x] - ca) + ed.lg_a[x] + (ed.lam_b[y] - cb) + ed.lg_b[y] - C / ed.eps);
  }
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
template <int DIM, int R, bool EXPL>
static hipError_t launch_msg_t(const Tables& tb, int n_items, int src_slot, hipStream_t s) {
  hipLaunchKernelGGL((k_msg<DIM, R, EXPL>), dim3(n_items), dim3(kBlock), 0, s, tb, src_slot);
  return hipGetLastError();
}

template <int R>
static hipError_t launch_msg_r(const Tables& tb, int n_items, int dim, int src_slot, hipStream_t s) {
  switch (dim) {
    case 0: return launch_msg_t<1, R, true>(tb, n_items, src_slot, s);  // explicit cost
    case 1: return launch_msg_t<1, R, false>(tb, n_items, src_slot, s);
    case 2: return launch_msg_t<2, R, false>(tb, n_items, src_slot, s);
    case 3: return launch_msg_t<3, R, false>(tb, n_items, src_slot, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_msg(const Tables& tb, int n_items, int dim, int rows_per_lane, int src_slot, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (src_slot < -1 || src_slot >= kSlots) return hipErrorInvalidValue;
  return rows_per_lane == 2 ? launch_msg_r<2>(tb, n_items, dim, src_slot, s)
                            : launch_msg_r<1>(tb, n_items, dim, src_slot, s);
}

template <int DIM, int W, int R, int H, bool F64, bool EXPL>
static hipError_t launch_node_t(const Tables& tb, int n_tiles, hipStream_t s) {
  hipLaunchKernelGGL((k_node<DIM, W, R, H, F64, EXPL>), dim3(n_tiles + tb.n_fin), dim3(64 * W), 0, s, tb);
  return hipGetLastError();
}

template <int W, int R, int H, bool F64>
static hipError_t launch_node_w(const Tables& tb, int n_tiles, int dim, hipStream_t s) {
  switch (dim) {
    case 0:  // explicit cost (one row per lane, one lane group only)
      if (R != 1 || H != 1) return hipErrorInvalidValue;
      return launch_node_t<1, W, 1, 1, F64, true>(tb, n_tiles, s);
    case 1: return launch_node_t<1, W, R, H, F64, false>(tb, n_tiles, s);
    case 2: return launch_node_t<2, W, R, H, F64, false>(tb, n_tiles, s);
    case 3: return launch_node_t<3, W, R, H, F64, false>(tb, n_tiles, s);
    default: return hipErrorInvalidValue;
  }
}

template <int R, int H>
static hipError_t launch_node_r(const Tables& tb, int n_tiles, int dim, int waves, bool fp64, hipStream_t s) {
  switch (waves) {
    case 2: return fp64 ? launch_node_w<2, R, H, true>(tb, n_tiles, dim, s) : launch_node_w<2, R, H, false>(tb, n_tiles, dim, s);
    case 4: return fp64 ? launch_node_w<4, R, H, true>(tb, n_tiles, dim, s) : launch_node_w<4, R, H, false>(tb, n_tiles, dim, s);
    case 8: return fp64 ? launch_node_w<8, R, H, true>(tb, n_tiles, dim, s) : launch_node_w<8, R, H, false>(tb, n_tiles, dim, s);
    case 16: return fp64 ? launch_node_w<16, R, H, true>(tb, n_tiles, dim, s) : launch_node_w<16, R, H, false>(tb, n_tiles, dim, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_node(const Tables& tb, int n_tiles, int dim, int waves, int rows_per_lane, int lane_groups,
                       bool fp64, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (rows_per_lane == 1 && lane_groups == 1) return launch_node_r<1, 1>(tb, n_tiles, dim, waves, fp64, s);
  // explicit-cost tiles take one row per lane and one lane group
  if (dim == 0) return hipErrorInvalidValue;
  if (rows_per_lane == 2 && lane_groups == 1) return launch_node_r<2, 1>(tb, n_tiles, dim, waves, fp64, s);
  if (rows_per_lane == 2 && lane_groups == 2) return launch_node_r<2, 2>(tb, n_tiles, dim, waves, fp64, s);
  if (rows_per_lane == 1 && lane_groups == 2) return launch_node_r<1, 2>(tb, n_tiles, dim, waves, fp64, s);
  return hipErrorInvalidValue;
}

hipError_t launch_finalize(const Tables& tb, int n_inst, hipStream_t s) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(n_inst), dim3(64 * kFinWaves), 0, s, tb);
  return hipGetLastError();
}

hipError_t launch_sep_pass(const Tables& tb, int pass, int n_items, size_t lds_bytes, bool fp64, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (lds_bytes > 64 * 1024) return hipErrorInvalidValue;
  if (pass == 0) {
    const dim3 grid(n_items + tb.n_fin);
    if (fp64) hipLaunchKernelGGL((k_sep_pass<true, 0>), grid, dim3(64 * kSepWaves), lds_bytes, s, tb);
    else hipLaunchKernelGGL((k_sep_pass<false, 0>), grid, dim3(64 * kSepWaves), lds_bytes, s, tb);
  } else {
    if (tb.n_fin != 0) return hipErrorInvalidValue;
    if (fp64) hipLaunchKernelGGL((k_sep_pass<true, 1>), dim3(n_items), dim3(64 * kSepWaves), lds_bytes, s, tb);
    else hipLaunchKernelGGL((k_sep_pass<false, 1>), dim3(n_items), dim3(64 * kSepWaves), lds_bytes, s, tb);
  }
  return hipGetLastError();
}

hipError_t launch_node_sep(const Tables& tb, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (tb.rec_rows != 32 && tb.rec_rows != 64) return hipErrorInvalidValue;
  const int waves = n_tiles * (64 / tb.rec_rows);
  hipLaunchKernelGGL(k_node_sep, dim3((waves + kSepWaves - 1) / kSepWaves), dim3(64 * kSepWaves), 0, s, tb,
                     n_tiles);
  return hipGetLastError();
}

hipError_t launch_msg_grid(const Tables& tb, int n_items, int rows_per_lane, bool eval, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (eval && tb.n_fin != 0) return hipErrorInvalidValue;
  const dim3 grid((n_items + kGridWaves - 1) / kGridWaves + tb.n_fin), block(64 * kGridWaves);
  if (rows_per_lane == 1) {
    if (eval) hipLaunchKernelGGL((k_msg_grid<1, true>), grid, block, 0, s, tb, n_items);
    else hipLaunchKernelGGL((k_msg_grid<1, false>), grid, block, 0, s, tb, n_items);
  } else if (rows_per_lane == 2) {
    if (eval) hipLaunchKernelGGL((k_msg_grid<2, true>), grid, block, 0, s, tb, n_items);
    else hipLaunchKernelGGL((k_msg_grid<2, false>), grid, block, 0, s, tb, n_items);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sep_horner(const Tables& tb, int pass, int n_tasks, bool eval, hipStream_t s) {
  if (n_tasks <= 0) return hipSuccess;
  const int blocks = (n_tasks + kSepWaves - 1) / kSepWaves;
  if ((pass == 1 || eval) && tb.n_fin != 0) return hipErrorInvalidValue;
  const dim3 block(64 * kSepWaves);
  if (pass == 0) {
    if (eval) hipLaunchKernelGGL((k_sep_horner<0, true>), dim3(blocks), block, 0, s, tb, n_tasks);
    else hipLaunchKernelGGL((k_sep_horner<0, false>), dim3(blocks + tb.n_fin), block, 0, s, tb, n_tasks);
  } else {
    if (eval) hipLaunchKernelGGL((k_sep_horner<1, true>), dim3(blocks), block, 0, s, tb, n_tasks);
    else hipLaunchKernelGGL((k_sep_horner<1, false>), dim3(blocks), block, 0, s, tb, n_tasks);
  }
  return hipGetLastError();
}

hipError_t launch_gs_update(const Tables& tb, int node_item, int slot, hipStream_t s) {
  if (node_item < 0 || slot < 0 || slot >= kSlots) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gs_update, dim3(1), dim3(kBlock), 0, s, tb, node_item, slot);
  return hipGetLastError();
}

hipError_t launch_node_eval(const Tables& tb, int n_nodes, int slot, hipStream_t s) {
  if (n_nodes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_node_eval, dim3(n_nodes), dim3(kBlock), 0, s, tb, slot);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_seg_copy(const SegCopy* segs) {
  const SegCopy sg = segs[blockIdx.x];
  const double c = sg.c ? *sg.c : 0.0;
  for (int64_t i = threadIdx.x; i < sg.len; i += kBlock) sg.dst[i] = sg.src[i] - c;
}

hipError_t launch_seg_copy(const SegCopy* segs, int n_segs, hipStream_t s) {
  if (n_segs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_seg_copy, dim3(n_segs), dim3(kBlock), 0, s, segs);
  return hipGetLastError();
}

hipError_t launch_zero_segs(const ZeroSeg* segs, int n_segs, hipStream_t s) {
  if (n_segs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_segs, dim3(n_segs), dim3(kBlock), 0, s, segs);
  return hipGetLastError();
}

hipError_t launch_stamp(InstState* inst, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stamp, dim3((count + kBlock - 1) / kBlock), dim3(kBlock), 0, s, inst, count);
  return hipGetLastError();
}

hipError_t launch_pairs(const EdgeDesc* edges, const PairItem* items, int n_items, double4* out, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pairs, dim3(n_items), dim3(kBlock), 0, s, edges, items, out);
  return hipGetLastError();
}

hipError_t launch_coupling(const EdgeDesc* edge, double* out, size_t total, hipStream_t s) {
  size_t blocks = (total + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_coupling, dim3((unsigned)blocks), dim3(kBlock), 0, s, edge, out);
  return hipGetLastError();
}

}  // namespace gmot
