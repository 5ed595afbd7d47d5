// gfx950 kernels of the bipartite iterative-scaling hot path.
//
//   k_msg<..., ITER>  -- message log-sum-exp m_{k->j} over a (row tile, column
//              split) of one message (the K u products of Theorem
//              tree_dual_var, eq. q).
//   k_tile     -- per 256-row tile of a node of the class: merge of the column
//              splits, stopping-sum terms of the state before the update
//              (Algorithm tree_local_reg; Lemma f_upper_bound_tree for the
//              arithmetic mean) and the update of eq. bipartite_tree_updates1/2
//              in its closed form (Proposition equi).
//   k_finalize -- per instance: node normalisers, stopping sum, stop decision.
//   k_msg<..., EVAL>  -- the same message LSE with given slots, no update.
//   k_node_eval       -- evaluation: merge, stopping-sum terms, <Lam, mu> / rho.
//   k_pairs           -- FP64 transport / entropy / mass sums of every plan
//                        (eq. bi-marginal_B_sol, eq. ot_graph_pairwise_mass).
//   k_coupling        -- one plan written out in FP64.
//
// Arithmetic contract of the FP32-core message kernel: FP64 potentials, FP64
// exponent arguments (w - row max), FP32 v_exp_f32 on the reduced argument,
// pairs of FP32 terms added in FP32 and accumulated in FP64, FP64 merge, log,
// stopping-sum terms and node normalisers.
#include "gmot_internal.h"

#include <cmath>

namespace gmot {

namespace {

constexpr int kRegDeg = 8;     // incident edges whose messages the tile kernel keeps in registers
constexpr int kRecChunk = 64;  // tile records reduced per block barrier
constexpr int kGroup = 4;      // edges whose loads the tile kernel issues together
constexpr int kNsReg = 8;      // column splits per edge held in registers by the tile kernel

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
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
    if (E < st->best_err) {
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
// Message log-sum-exp.  Block = 4 waves; lane l of wave w owns rows
// row0 + (w*R + r)*64 + l, r < R.  Columns are streamed through LDS in chunks.
// Output per row and column split: (M, sum 2^(w - M)) with M the split's max.
//
// Two passes (first computations, FP64 path, evaluation): per chunk, pass 1
// finds the row max and pass 2 sums 2^(w - max); the running sum is rescaled
// when the max grows.
// One pass (FP32-core iteration from the third half-sweep of a call on): the
// shift s is the max of the same row and column split at the previous
// computation of the message (still in the partial buffer), and one pass sums
// 2^(w - s) while tracking the max.  Any finite s gives the
// exact sum while the terms stay in FP32 range; a chunk whose max exceeds s by
// more than kShiftHi moves s up to that max and is summed again, and if a
// row's max ends more than kShiftLo below s (its top terms would lose FP32
// precision) the block repeats its columns in two passes.  Both decisions are
// block-uniform.  Near convergence s differs from the max by the drift of the
// iteration, so the dominant terms' arguments are nearly exact, as in two passes.
// ITER: slots come from the instance counter; finished instances (or those
// whose next half-sweep updates the other class) return at entry.
// ---------------------------------------------------------------------------
constexpr double kShiftHi = 96.0;
constexpr double kShiftLo = -96.0;

template <int DIM, int R, bool F64, bool EXPL, bool ITER>
__global__ __launch_bounds__(kBlock) void k_msg(Tables tb, int eval_src_slot) {
  constexpr int CH = EXPL ? 32 : kChunk;            // columns per LDS chunk
  constexpr int STR = EXPL ? 1 : (DIM == 1 ? 2 : 4); // doubles per staged column
  constexpr int TM = 256 * R;                        // rows per block
  __shared__ double s_col[CH * STR];
  __shared__ float s_cost[EXPL ? CH * TM : 1];

  const K1Item it = tb.items[blockIdx.x];
  const MsgDesc* __restrict__ md = tb.msgs + it.msg;
  int src_slot = eval_src_slot;
  bool one = false;
  if (ITER) {
    const InstState* st = tb.inst + it.inst;
    const long long t = st->t;
    if (st->done || ((t & 1) == 1) != (tb.colour == 0)) return;
    src_slot = (int)((t >> 1) & 1);
    one = !F64 && t >= st->onepass_from;
  }
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
  double s0[R];  // one-pass shift from the previous computation
#pragma unroll
  for (int r = 0; r < R; ++r) {
    row[r] = it.row0 + (wave * R + r) * 64 + lane;
    const bool v = row[r] < n_dst;
#pragma unroll
    for (int d = 0; d < DIM; ++d) cx[r][d] = (v && !EXPL) ? cxs * md->supp_dst[(size_t)row[r] * DIM + d] : 0.0;
    s0[r] = 0.0;
    if (one && v) {
      const double m = md->partial[(size_t)row[r] * md->ns + it.split].x;
      s0[r] = isfinite(m) ? m : 0.0;
    }
  }

  // w(x, y) of local row slot (wave*R + r) and staged column c
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
  // sum of 2^(w - sh) over the staged chunk (pairs of FP32 terms, FP64 accumulation)
  auto chunk_sum = [&](int cpad, const double* sh, double* out) {
#pragma unroll
    for (int r = 0; r < R; ++r) out[r] = 0.0;
#pragma unroll 4
    for (int c = 0; c < cpad; c += 2) {
      const double a0 = s_col[c * STR];
      const double a1 = s_col[(c + 1) * STR];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double w0 = wval(r, c, a0), w1 = wval(r, c + 1, a1);
        if (F64) {
          out[r] += exp2(w0 - sh[r]) + exp2(w1 - sh[r]);
        } else {
          const float p = exp2_hw((float)(w0 - sh[r])) + exp2_hw((float)(w1 - sh[r]));
          out[r] += (double)p;
        }
      }
    }
  };

  double Mrun[R], Srun[R], shift[R];
  for (int attempt = 0; attempt < 2; ++attempt) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      Mrun[r] = -INFINITY;
      Srun[r] = 0.0;
      shift[r] = s0[r];
    }
    for (int c0 = 0; c0 < it.ncols; c0 += CH) {
      const int cn = min(CH, it.ncols - c0);
      const int cpad = (cn + 7) & ~7;
      __syncthreads();  // previous chunk fully consumed
      if (threadIdx.x < cpad) {
        double a = -INFINITY;
        double y[DIM > 0 ? DIM : 1];
#pragma unroll
        for (int d = 0; d < DIM; ++d) y[d] = 0.0;
        if (threadIdx.x < cn) {
          const int col = it.col0 + c0 + threadIdx.x;
          double base = (lam[col] - csrc) + lg[col];
          if (!EXPL) {
            double y2 = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
              y[d] = ys[(size_t)col * DIM + d];
              y2 = fma(y[d], y[d], y2);
            }
            base -= y2 / eps;
          }
          a = kLog2e * base;
        }
        s_col[threadIdx.x * STR] = a;
        if (!EXPL) {
#pragma unroll
          for (int d = 0; d < DIM; ++d) s_col[threadIdx.x * STR + 1 + d] = y[d];
        }
      }
      if (EXPL) {
        // cost tile, stored src-major: cost[y * n_dst + x]; coalesced over x
        for (int c = 0; c < cpad; ++c) {
          const int col = it.col0 + c0 + c;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int lr = r * 256 + threadIdx.x;
            const int x = it.row0 + lr;
            float v = 0.0f;
            if (c < cn && x < n_dst) v = md->cost[(size_t)col * n_dst + x];
            s_cost[c * TM + lr] = v;
          }
        }
      }
      __syncthreads();

      if (one) {
        // one pass: sum relative to the shift, chunk max alongside
        double Mc[R], Sc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          Mc[r] = -INFINITY;
          Sc[r] = 0.0;
        }
#pragma unroll 4
        for (int c = 0; c < cpad; c += 2) {
          const double a0 = s_col[c * STR];
          const double a1 = s_col[(c + 1) * STR];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const double w0 = wval(r, c, a0), w1 = wval(r, c + 1, a1);
            Mc[r] = fmax(Mc[r], fmax(w0, w1));
            const float p = exp2_hw((float)(w0 - shift[r])) + exp2_hw((float)(w1 - shift[r]));
            Sc[r] += (double)p;
          }
        }
        int hi = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          Mrun[r] = fmax(Mrun[r], Mc[r]);
          if (row[r] < n_dst && Mc[r] - shift[r] > kShiftHi) hi = 1;
        }
        if (__syncthreads_or(hi)) {
          // move the shift of far-exceeded rows up to the chunk max and sum again
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if (Mc[r] - shift[r] > kShiftHi) {
              Srun[r] *= exp2(shift[r] - Mc[r]);
              shift[r] = Mc[r];
            }
          }
          chunk_sum(cpad, shift, Sc);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) Srun[r] += Sc[r];
      } else {
        // pass 1: chunk max per row
        double Mc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) Mc[r] = -INFINITY;
#pragma unroll 8
        for (int c = 0; c < cpad; ++c) {
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
          shift[r] = (Mrun[r] == -INFINITY) ? 0.0 : Mrun[r];
        }
        // pass 2: sum of 2^(w - max)
        double Sc[R];
        chunk_sum(cpad, shift, Sc);
#pragma unroll
        for (int r = 0; r < R; ++r) Srun[r] += Sc[r];
      }
    }
    if (!one) break;
    // one pass: express the sum relative to the split max; rows whose max fell
    // far below the shift send the block back through its columns in two passes
    int lo = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (row[r] < n_dst && Mrun[r] > -INFINITY && Mrun[r] - shift[r] < kShiftLo) lo = 1;
    if (__syncthreads_or(lo)) {
      one = false;
      continue;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (Mrun[r] > -INFINITY) {
        Srun[r] *= exp2(shift[r] - Mrun[r]);
      } else {
        Srun[r] = 0.0;
      }
    }
    break;
  }

#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (row[r] < n_dst) md->partial[(size_t)row[r] * md->ns + it.split] = make_double2(Mrun[r], Srun[r]);
  }
}

// ---------------------------------------------------------------------------
// Tile kernel: one thread per row x of a 256-row tile of node j.
//   merge  m_{k->j}(x) from the column splits (FP64)
//   terms  fixed:  mu(x) |expm1(Lam_(j,k)(x) + m_{k->j}(x))| = |q_(j,k)(x) - mu(x)|
//          free:   |q_(j,k)(x) - qbar(x)|, q = exp(Lam + m), qbar the mean over k
//   update fixed:  L_(j,k) = -m_{k->j}        (c_j = 0)
//          free:   L_(j,k) = abar - m_{k->j}  (abar = mean_k m; c_j = LSE_x abar
//                  is formed by the finalise kernel from the tile records)
// Record: per incident edge the tile's sum of terms, then the tile's LSE of
// abar (max, scaled sum).
// The loads of a group of kGroup edges (descriptors, split partials, held
// potentials) are issued together, so a tile waits for memory once per group
// rather than several times per edge.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_tile(Tables tb) {
  __shared__ double sh_rec[4][kRecChunk + kRecExtra];
  const TileItem ti = tb.tiles[blockIdx.x];
  const InstState* st = tb.inst + ti.inst;
  const NodeItem nd = tb.nodes[ti.node];
  const long long t = st->t;
  if (st->done || ((t & 1) == 1) != (tb.colour == 0)) return;
  const int cur = (int)(((t - 1) >> 1) & 1), nxt = cur ^ 1;
  const MsgDesc* __restrict__ mds = tb.msgs + nd.msg0;
  const int n = nd.n, deg = nd.deg;
  const bool fixed = nd.fixed != 0;
  const int dim = mds[0].dim;
  const bool sq = mds[0].cost_kind == 0;
  const double ieps = 1.0 / mds[0].eps;
  const double* __restrict__ xs = mds[0].supp_dst;
  const double c_old = nd.c ? nd.c[cur] : 0.0;
  double* __restrict__ rec = nd.tpart + (size_t)(ti.row0 / kTileRows) * (deg + kRecExtra);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = ti.row0 + threadIdx.x;
  const bool vx = x < n;
  const double mux = (vx && fixed) ? nd.mu[x] : 0.0;
  const double x2 = (vx && sq) ? sq_norm(xs, dim, x) : 0.0;

  // merged messages and held potentials: registers for the first kRegDeg
  // edges, the mfull scratch row beyond (star centres of high degree)
  double mreg[kRegDeg], lreg[kRegDeg];
  double asum = 0.0, qsum = 0.0;
  auto finish = [&](const MsgDesc& md, const Merged& g, double l) -> double {
    const double m = (g.lse2 > -INFINITY) ? kLn2 * g.lse2 - x2 * ieps : -INFINITY;
    asum += m;
    if (!fixed) qsum += exp(l - c_old + m);
    return m;
  };
#pragma unroll
  for (int g0 = 0; g0 < kRegDeg; g0 += kGroup) {
    const double2* P[kGroup];
    const double* Lc[kGroup];
    int NS[kGroup];
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      const bool on = g0 + u < deg;
      P[u] = on ? mds[g0 + u].partial : nullptr;
      Lc[u] = on ? mds[g0 + u].lam_dst[cur] : nullptr;
      NS[u] = on ? mds[g0 + u].ns : 0;
    }
    double2 pv[kGroup][kNsReg];
    double lv[kGroup];
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      const bool on = vx && g0 + u < deg;
      lv[u] = on ? Lc[u][x] : 0.0;
#pragma unroll
      for (int s2 = 0; s2 < kNsReg; ++s2)
        pv[u][s2] = (on && s2 < NS[u]) ? P[u][(size_t)x * NS[u] + s2] : make_double2(-INFINITY, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      const int k = g0 + u;
      mreg[k] = 0.0;
      lreg[k] = lv[u];
      if (k < deg && vx) {
        Merged g;
        if (NS[u] <= kNsReg) {
          double Mx = -INFINITY;
#pragma unroll
          for (int s2 = 0; s2 < kNsReg; ++s2) Mx = fmax(Mx, pv[u][s2].x);
          double S = 0.0;
          if (Mx > -INFINITY) {
#pragma unroll
            for (int s2 = 0; s2 < kNsReg; ++s2) {
              const double2 q = pv[u][s2];
              if (q.y > 0.0) S += (q.x == Mx) ? q.y : q.y * exp2(q.x - Mx);
            }
          }
          g = {(S > 0.0) ? Mx + log2(S) : -INFINITY, Mx, S};
        } else {
          g = merge_splits(P[u] + (size_t)x * NS[u], NS[u]);
        }
        mreg[k] = finish(mds[k], g, lv[u]);
      }
    }
  }
  for (int k = kRegDeg; k < deg; ++k) {
    if (!vx) continue;
    const MsgDesc& md = mds[k];
    const Merged g = merge_splits(md.partial + (size_t)x * md.ns, md.ns);
    md.mfull[x] = finish(md, g, md.lam_dst[cur][x]);
  }
  const double a = vx ? asum / deg : -INFINITY;
  const double qb = qsum / deg;

  // stopping-sum term of edge k at row x, and the update of L_(j,k)(x)
  auto term = [&](int k, double m, double l) -> double {
    double part = 0.0;
    if (vx) {
      double* __restrict__ Ln = mds[k].lam_dst[nxt];
      if (fixed) {
        if (mux > 0.0) part = mux * fabs(expm1(l + m));
        Ln[x] = -m;
      } else {
        part = fabs(exp(l - c_old + m) - qb);
        Ln[x] = a - m;
      }
    }
    return wave_sum(part);
  };

  // records in chunks of kRecChunk edges, one barrier per chunk
  for (int k0 = 0; k0 < deg; k0 += kRecChunk) {
    const int kn = min(kRecChunk, deg - k0);
    if (k0 == 0) {
#pragma unroll
      for (int k = 0; k < kRegDeg; ++k) {
        if (k < kn) {
          const double p = term(k, mreg[k], lreg[k]);
          if (lane == 0) sh_rec[wave][k] = p;
        }
      }
    }
    for (int k = max(k0, kRegDeg); k < k0 + kn; ++k) {
      const double m = vx ? mds[k].mfull[x] : 0.0;
      const double l = vx ? mds[k].lam_dst[cur][x] : 0.0;
      const double p = term(k, m, l);
      if (lane == 0) sh_rec[wave][k - k0] = p;
    }
    const bool last = k0 + kn == deg;
    if (last && !fixed) {
      // per-wave LSE of abar over the wave's rows
      const double Mw = wave_max(a);
      const double Sw = wave_sum((a > -INFINITY) ? exp(a - Mw) : 0.0);
      if (lane == 0) {
        sh_rec[wave][kn] = Mw;
        sh_rec[wave][kn + 1] = Sw;
      }
    }
    __syncthreads();
    const int i = threadIdx.x;
    if (i < kn) rec[k0 + i] = (sh_rec[0][i] + sh_rec[1][i]) + (sh_rec[2][i] + sh_rec[3][i]);
    if (last && !fixed && i == kn) {
      double M = -INFINITY;
      for (int w = 0; w < 4; ++w) M = fmax(M, sh_rec[w][kn]);
      double S = 0.0;
      for (int w = 0; w < 4; ++w)
        if (sh_rec[w][kn] > -INFINITY) S += sh_rec[w][kn + 1] * exp(sh_rec[w][kn] - M);
      rec[deg] = M;
      rec[deg + 1] = S;
    }
    if (!last) __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Finalise kernel: one block per instance.  Thread i handles the instance's
// class nodes i, i + 256, ...: per-edge terms summed over tiles (the node's
// stopping-sum terms), and for free nodes c_j = LSE over the tile records;
// then the block sums the terms and thread 0 takes the stop decision.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_finalize(Tables tb) {
  __shared__ double sh[4][2];
  InstState* st = tb.inst + blockIdx.x;
  const long long t = st->t;
  if (st->done || ((t & 1) == 1) != (tb.colour == 0)) return;
  const int nxt = (int)((((t - 1) >> 1) & 1) ^ 1);
  const int i0 = st->node0[tb.colour], cnt = st->nnodes[tb.colour];
  double esum = 0.0, emax = 0.0;
  for (int i = threadIdx.x; i < cnt; i += kBlock) {
    const NodeItem nd = tb.nodes[i0 + i];
    const int deg = nd.deg, stride = deg + kRecExtra, tiles = nd.tiles;
    const double* __restrict__ tp = nd.tpart;
    for (int k = 0; k < deg; ++k) {
      double e = 0.0;
      for (int tt = 0; tt < tiles; ++tt) e += tp[(size_t)tt * stride + k];
      esum += e;
      emax = fmax(emax, e);
    }
    if (!nd.fixed) {
      double M = -INFINITY;
      for (int tt = 0; tt < tiles; ++tt) M = fmax(M, tp[(size_t)tt * stride + deg]);
      double S = 0.0;
      for (int tt = 0; tt < tiles; ++tt) {
        const double mt = tp[(size_t)tt * stride + deg];
        if (mt > -INFINITY) S += tp[(size_t)tt * stride + deg + 1] * exp(mt - M);
      }
      nd.c[nxt] = M + log(S);
    }
  }
  esum = wave_sum(esum);
  emax = wave_max(emax);
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x >> 6][0] = esum;
    sh[threadIdx.x >> 6][1] = emax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double E = (sh[0][0] + sh[1][0]) + (sh[2][0] + sh[3][0]);
    const double Em = fmax(fmax(sh[0][1], sh[1][1]), fmax(sh[2][1], sh[3][1]));
    decide(tb, st, t, E, Em);
  }
}

// ---------------------------------------------------------------------------
// Evaluation node pass (one block per node, given slot): merge the splits,
// stopping-sum terms of the state, qbar (the node marginal q_bar_j), and
// <Lam, mu> (constrained) or rho_j and its spread in x (free).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_node_eval(Tables tb, int slot) {
  __shared__ double sh[4];
  const NodeItem nd = tb.nodes[blockIdx.x];
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
    double part = 0.0;
    for (int x = threadIdx.x; x < n; x += kBlock) {
      const double q = exp(md.lam_dst[slot][x] - cj + nd.lg[x] + md.mfull[x]);
      const double ref = nd.fixed ? nd.mu[x] : nd.qbar[x];
      part += fabs(q - ref);
    }
    const double tot = block_sum(part, sh);
    e_sum += tot;
    e_max = fmax(e_max, tot);
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

// ---------------------------------------------------------------------------
// FP64 pair pass: for each plan, sum_xy C B, sum_xy B (log B - log M - 1)
// and sum_xy B over a (256 rows x ncols) tile.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_pairs(const EdgeDesc* edges, const PairItem* items, double4* out) {
  __shared__ double sh[4];
  __shared__ double s_b[kChunk];
  __shared__ double s_y[kChunk * 3];
  const PairItem it = items[blockIdx.x];
  const EdgeDesc ed = edges[it.edge];
  const int x = it.row0 + threadIdx.x;
  const bool vx = x < ed.n_a;
  const bool sq = ed.cost_kind == 0;
  const double ca = ed.c_a ? *ed.c_a : 0.0;
  const double cb = ed.c_b ? *ed.c_b : 0.0;
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
        const double lgb = ed.lg_b[y];
        const double lb = s_b[c];
        const double logB = ax + lb + lgb - C / ed.eps;
        const double B = exp(logB);
        if (B > 0.0) {
          sT += C * B;
          sH += B * (lax + lb - C / ed.eps - 1.0);
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
template <int DIM, int R, bool F64, bool EXPL>
static hipError_t launch_msg_t(const Tables& tb, int n_items, int eval_src_slot, hipStream_t s) {
  if (eval_src_slot >= 0)
    hipLaunchKernelGGL((k_msg<DIM, R, F64, EXPL, false>), dim3(n_items), dim3(kBlock), 0, s, tb, eval_src_slot);
  else
    hipLaunchKernelGGL((k_msg<DIM, R, F64, EXPL, true>), dim3(n_items), dim3(kBlock), 0, s, tb, -1);
  return hipGetLastError();
}

template <int R, bool F64>
static hipError_t launch_msg_r(const Tables& tb, int n_items, int dim, int eval_src_slot, hipStream_t s) {
  switch (dim) {
    case 0: return launch_msg_t<1, R, F64, true>(tb, n_items, eval_src_slot, s);  // explicit cost
    case 1: return launch_msg_t<1, R, F64, false>(tb, n_items, eval_src_slot, s);
    case 2: return launch_msg_t<2, R, F64, false>(tb, n_items, eval_src_slot, s);
    case 3: return launch_msg_t<3, R, F64, false>(tb, n_items, eval_src_slot, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_msg(const Tables& tb, int n_items, int dim, int rows_per_lane, bool fp64, int eval_src_slot,
                      hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (rows_per_lane == 2) {
    return fp64 ? launch_msg_r<2, true>(tb, n_items, dim, eval_src_slot, s)
                : launch_msg_r<2, false>(tb, n_items, dim, eval_src_slot, s);
  }
  return fp64 ? launch_msg_r<1, true>(tb, n_items, dim, eval_src_slot, s)
              : launch_msg_r<1, false>(tb, n_items, dim, eval_src_slot, s);
}

hipError_t launch_tile(const Tables& tb, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile, dim3(n_tiles), dim3(kBlock), 0, s, tb);
  return hipGetLastError();
}

hipError_t launch_finalize(const Tables& tb, int n_inst, hipStream_t s) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(n_inst), dim3(kBlock), 0, s, tb);
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
