// Rounding of the plans onto the constraint set (Algorithm round).
//
// After a half-sweep, the class S that was not updated last misses its
// marginals.  For every edge, with j its end in S and k the other end, the plan
// B = B_(j,k) (rows on j) is rounded with the rounding of Altschuler, Weed and
// Rigollet onto the polytope whose row marginal is r (mu_j for a constrained
// node, the arithmetic mean q_bar_j of the node's plan marginals for a free
// one) and whose column marginal is c = B^T 1, which is already consistent at
// k because k was updated last:
//     X = min(r / B1, 1),  Y = min(c / (XB)^T 1, 1),  F = diag(X) B diag(Y),
//     e_r = r - F1 >= 0,   e_c = c - F^T 1 >= 0,      G = F + e_r e_c^T / |e_r|_1.
// Nothing of size n_j x n_k is stored: three FP64 row passes over recomputed
// plan entries give the scalings, the residuals and the rounded transport
//     <C, G> = sum_x X(x) sum_y B(x,y) Y(y) C(x,y) + (e_r^T C e_c) / |e_r|_1,
// and G itself is written out only on request.
//
//   pass 0 (every directed edge, rows on its first node): row sums B1.
//   node kernel (nodes of S): r, X for every incident edge, and the node's
//          term of the stopping sum (the parenthesis of Lemma round).
//   pass 1 (rows on k): (XB)^T 1, then Y and e_c.
//   pass 2 (rows on j): F1 = X (B Y), e_r, and the block's share of both
//          transport terms.
#include "gmot_internal.h"

#include <cmath>

namespace gmot {

namespace {

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

}  // namespace

template <int PASS>
__global__ __launch_bounds__(kBlock) void k_round_rows(const RoundDesc* ds, const RoundItem* items, double4* part) {
  __shared__ double s_b[kChunk], s_w[kChunk], s_e[kChunk], s_y[kChunk * 3];
  __shared__ double sh[4][4];
  const RoundItem it = items[blockIdx.x];
  const RoundDesc d = ds[it.desc];
  const int x = it.row0 + threadIdx.x;
  const bool vx = x < d.n_r;
  const bool sq = d.cost_kind == 0;
  const double cj = d.c_r ? *d.c_r : 0.0;
  const double ck = d.c_c ? *d.c_c : 0.0;
  double la = -INFINITY, xp[3] = {0.0, 0.0, 0.0};
  if (vx) {
    la = (d.lam_r[x] - cj) + d.lg_r[x];
    if (sq)
      for (int k = 0; k < d.dim; ++k) xp[k] = d.supp_r[(size_t)x * d.dim + k];
  }
  double g = 0.0, gc = 0.0, h = 0.0, cmax = 0.0;
  for (int c0 = 0; c0 < d.n_c; c0 += kChunk) {
    const int cn = min(kChunk, d.n_c - c0);
    __syncthreads();
    if (threadIdx.x < cn) {
      const int y = c0 + threadIdx.x;
      s_b[threadIdx.x] = (d.lam_c[y] - ck) + d.lg_c[y];
      s_w[threadIdx.x] = d.sc_col ? d.sc_col[y] : 1.0;
      if (PASS == 2) s_e[threadIdx.x] = d.er_col[y];
      if (sq)
        for (int k = 0; k < d.dim; ++k) s_y[threadIdx.x * 3 + k] = d.supp_c[(size_t)y * d.dim + k];
    }
    __syncthreads();
    if (vx) {
      for (int c = 0; c < cn; ++c) {
        double C;
        if (sq) {
          C = 0.0;
          for (int k = 0; k < d.dim; ++k) {
            const double df = xp[k] - s_y[c * 3 + k];
            C = fma(df, df, C);
          }
        } else {
          C = (double)d.cost[(size_t)(c0 + c) * d.n_r + x];
        }
        const double bw = exp(la + s_b[c] - C / d.eps) * s_w[c];
        g += bw;
        if (PASS == 2) {
          gc += bw * C;
          h += C * s_e[c];
          cmax = fmax(cmax, fabs(C));
        }
      }
    }
  }
  if (PASS == 0) {
    if (vx) d.rs[x] = g;
    return;
  }
  if (PASS == 1) {
    if (vx) {
      const double c = d.rs[x];
      const double Y = g > 0.0 ? fmin(c / g, 1.0) : 1.0;
      d.sc[x] = Y;
      d.er[x] = c - Y * g;
    }
    return;
  }
  double pt = 0.0, pb = 0.0, pe = 0.0;
  if (vx) {
    const double X = d.sc[x];
    const double e = d.tg[x] - X * g;
    d.er[x] = e;
    pt = X * gc;
    pb = e * h;
    pe = e;
  }
  pt = wsum(pt);
  pb = wsum(pb);
  pe = wsum(pe);
  cmax = wmax(cmax);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[w][0] = pt;
    sh[w][1] = pb;
    sh[w][2] = pe;
    sh[w][3] = cmax;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    part[blockIdx.x] = make_double4((sh[0][0] + sh[1][0]) + (sh[2][0] + sh[3][0]),
                                    (sh[0][1] + sh[1][1]) + (sh[2][1] + sh[3][1]),
                                    (sh[0][2] + sh[1][2]) + (sh[2][2] + sh[3][2]),
                                    fmax(fmax(sh[0][3], sh[1][3]), fmax(sh[2][3], sh[3][3])));
}

// One block per node j of S: row target r (mu_j, or the mean of the plan
// marginals over the node's edges), X = min(r / B1, 1) per edge, and the
// node's stopping-sum term sum_k |r - B_(j,k) 1|_1.
__global__ __launch_bounds__(kBlock) void k_round_node(const RoundNode* nodes, const RoundDesc* ds, double* err) {
  __shared__ double sh[4];
  const RoundNode nd = nodes[blockIdx.x];
  const RoundDesc* __restrict__ dj = ds + nd.d0;
  double e = 0.0;
  for (int x = threadIdx.x; x < nd.n; x += kBlock) {
    double r;
    if (nd.mu) {
      r = nd.mu[x];
    } else {
      r = 0.0;
      for (int k = 0; k < nd.deg; ++k) r += dj[k].rs[x];
      r /= nd.deg;
    }
    for (int k = 0; k < nd.deg; ++k) {
      const double rs = dj[k].rs[x];
      dj[k].tg[x] = r;
      dj[k].sc[x] = rs > 0.0 ? fmin(r / rs, 1.0) : 1.0;
      e += fabs(r - rs);
    }
  }
  e = wsum(e);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) err[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// The rounded plan G of one edge written as n_a x n_b row-major (a = the
// edge's first node); `d` is the directed edge with rows on the node in S,
// `o` its opposite.  s_is_a: the node in S is a.
__global__ __launch_bounds__(kBlock) void k_round_plan(const RoundDesc* dd, const RoundDesc* od, double inv_s,
                                                       int s_is_a, double* out) {
  const RoundDesc d = *dd;
  const RoundDesc o = *od;
  const double cj = d.c_r ? *d.c_r : 0.0;
  const double ck = d.c_c ? *d.c_c : 0.0;
  const size_t total = (size_t)d.n_r * d.n_c;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (size_t)gridDim.x * kBlock) {
    int x, y;  // x on j (rows of d), y on k
    if (s_is_a) {
      x = (int)(i / d.n_c);
      y = (int)(i % d.n_c);
    } else {
      y = (int)(i / d.n_r);
      x = (int)(i % d.n_r);
    }
    double C;
    if (d.cost_kind == 0) {
      C = 0.0;
      for (int k = 0; k < d.dim; ++k) {
        const double df = d.supp_r[(size_t)x * d.dim + k] - d.supp_c[(size_t)y * d.dim + k];
        C = fma(df, df, C);
      }
    } else {
      C = (double)d.cost[(size_t)y * d.n_r + x];
    }
    const double B = exp((d.lam_r[x] - cj) + d.lg_r[x] + (d.lam_c[y] - ck) + d.lg_c[y] - C / d.eps);
    out[i] = d.sc[x] * B * o.sc[y] + d.er[x] * o.er[y] * inv_s;
  }
}

hipError_t launch_round_rows(int pass, const RoundDesc* ds, const RoundItem* items, int n_items, double4* part,
                             hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  switch (pass) {
    case 0: hipLaunchKernelGGL(k_round_rows<0>, dim3(n_items), dim3(kBlock), 0, s, ds, items, part); break;
    case 1: hipLaunchKernelGGL(k_round_rows<1>, dim3(n_items), dim3(kBlock), 0, s, ds, items, part); break;
    case 2: hipLaunchKernelGGL(k_round_rows<2>, dim3(n_items), dim3(kBlock), 0, s, ds, items, part); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_round_node(const RoundNode* nodes, int n_nodes, const RoundDesc* ds, double* err, hipStream_t s) {
  if (n_nodes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_round_node, dim3(n_nodes), dim3(kBlock), 0, s, nodes, ds, err);
  return hipGetLastError();
}

hipError_t launch_round_plan(const RoundDesc* d, const RoundDesc* o, double inv_s, int s_is_a, double* out,
                             size_t total, hipStream_t s) {
  size_t blocks = (total + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_round_plan, dim3((unsigned)blocks), dim3(kBlock), 0, s, d, o, inv_s, s_is_a, out);
  return hipGetLastError();
}

}  // namespace gmot
