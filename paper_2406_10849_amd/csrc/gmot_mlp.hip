// Learned warm start: a small fully connected network trained on the GPU by
// these kernels (BF16 MFMA GEMMs with FP32 accumulation, FP32 master weights
// and Adam), plus the data movement between star instances and the network.
// The network is not part of the paper's method; it only initialises the
// potentials of the bipartite iteration, which still decides convergence.
#include "gmot.h"
#include "gmot_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

namespace gmot {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline double block_sum_d(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

}  // namespace

// ---------------------------------------------------------------------------
// GEMM  C[m][n] = sum_k A(m,k) B(k,n), BF16 inputs, FP32 accumulation on
// v_mfma_f32_16x16x32_bf16.  A(m,k) = TA ? A[k*lda+m] : A[m*lda+k];
// B(k,n) = TB ? B[n*ldb+k] : B[k*ldb+n].  M, N, K, lda, ldb multiples of 8.
// Block: 4 waves, 64x64 macro tile, each wave 32x32 = 2x2 MFMA tiles; K in
// steps of 32 staged through LDS with k contiguous per row / column.
// ---------------------------------------------------------------------------
enum Epi : int { kStore = 0, kBiasRelu = 1, kBias = 2, kMaskRelu = 3 };

struct GemmArgs {
  const uint16_t* A;
  const uint16_t* B;
  int M, N, K, lda, ldb, ldc;
  float* C;             // FP32 output (row-major, ldc)
  uint16_t* Cq;         // optional BF16 copy of the output (same layout)
  const float* bias;    // [N] for kBias / kBiasRelu
  const float* mask;    // [M x ldc] for kMaskRelu: multiply by (mask > 0)
  float* part;          // split-K: [gridDim.z x M x ldc] raw partial sums (no epilogue), or NULL
  int k_chunk;          // split-K: K values per split (a multiple of 32)
};

// The next K step's A and B chunks are loaded into registers while the
// current step's MFMAs run (one LDS buffer, two barriers per step).  With
// split-K (g.part set) block z sums K range [z k_chunk, (z + 1) k_chunk) and
// writes its raw partial sums; k_gemm_reduce adds the splits in order and
// applies the epilogue.
template <int EPI>
__device__ inline void gemm_epilogue(const GemmArgs& g, int m, int n, float v) {
  const size_t o = (size_t)m * g.ldc + n;
  if (EPI == kBias || EPI == kBiasRelu) v += g.bias[n];
  if (EPI == kBiasRelu) v = fmaxf(v, 0.f);
  if (EPI == kMaskRelu) v = g.mask[o] > 0.f ? v : 0.f;
  g.C[o] = v;
  if (g.Cq) g.Cq[o] = to_bf16(v);
}

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  constexpr int LDK = 40;  // 32 k values + 8 padding, rows stay 16-byte aligned
  __shared__ __attribute__((aligned(16))) uint16_t As[64 * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[64 * LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int kb = g.part ? (int)blockIdx.z * g.k_chunk : 0;
  const int ke = g.part ? min(g.K, kb + g.k_chunk) : g.K;
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  // this thread's 8-element chunks of A and B at K step k0 (zeros past the edges)
  auto load_a = [&](int k0) -> uint4 {
    uint4 v = make_uint4(0, 0, 0, 0);
    if (!TA) {
      const int m = m0 + (tid >> 2), k = k0 + (tid & 3) * 8;
      if (m < g.M && k < ke) v = *reinterpret_cast<const uint4*>(g.A + (size_t)m * g.lda + k);
    } else {
      const int kk = k0 + (tid >> 3), m = m0 + (tid & 7) * 8;
      if (kk < ke && m < g.M) v = *reinterpret_cast<const uint4*>(g.A + (size_t)kk * g.lda + m);
    }
    return v;
  };
  auto load_b = [&](int k0) -> uint4 {
    uint4 v = make_uint4(0, 0, 0, 0);
    if (TB) {
      const int n = n0 + (tid >> 2), k = k0 + (tid & 3) * 8;
      if (n < g.N && k < ke) v = *reinterpret_cast<const uint4*>(g.B + (size_t)n * g.ldb + k);
    } else {
      const int kk = k0 + (tid >> 3), n = n0 + (tid & 7) * 8;
      if (kk < ke && n < g.N) v = *reinterpret_cast<const uint4*>(g.B + (size_t)kk * g.ldb + n);
    }
    return v;
  };
  auto store_a = [&](uint4 v) {
    if (!TA) {
      *reinterpret_cast<uint4*>(&As[(tid >> 2) * LDK + (tid & 3) * 8]) = v;
    } else {
      const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
      const int k = tid >> 3, mc = (tid & 7) * 8;
#pragma unroll
      for (int i = 0; i < 8; ++i) As[(mc + i) * LDK + k] = e[i];
    }
  };
  auto store_b = [&](uint4 v) {
    if (TB) {
      *reinterpret_cast<uint4*>(&Bs[(tid >> 2) * LDK + (tid & 3) * 8]) = v;
    } else {
      const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
      const int k = tid >> 3, nc = (tid & 7) * 8;
#pragma unroll
      for (int i = 0; i < 8; ++i) Bs[(nc + i) * LDK + k] = e[i];
    }
  };

  uint4 ra = load_a(kb), rb = load_b(kb);
  for (int k0 = kb; k0 < ke; k0 += 32) {
    store_a(ra);
    store_b(rb);
    __syncthreads();
    if (k0 + 32 < ke) {
      ra = load_a(k0 + 32);
      rb = load_b(k0 + 32);
    }
#pragma unroll
    for (int sm = 0; sm < 2; ++sm)
#pragma unroll
      for (int sn = 0; sn < 2; ++sn) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[(wm + sm * 16 + (lane & 15)) * LDK + (lane >> 4) * 8]);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[(wn + sn * 16 + (lane & 15)) * LDK + (lane >> 4) * 8]);
        acc[sm][sn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[sm][sn], 0, 0, 0);
      }
    __syncthreads();
  }

#pragma unroll
  for (int sm = 0; sm < 2; ++sm)
#pragma unroll
    for (int sn = 0; sn < 2; ++sn)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = m0 + wm + sm * 16 + (lane >> 4) * 4 + i;
        const int n = n0 + wn + sn * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        if (g.part) g.part[((size_t)blockIdx.z * g.M + m) * g.ldc + n] = acc[sm][sn][i];
        else gemm_epilogue<EPI>(g, m, n, acc[sm][sn][i]);
      }
}

// Split-K: the splits of every output added in split order, then the epilogue.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_reduce(GemmArgs g, int splits) {
  const size_t total = (size_t)g.M * g.N;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (size_t)gridDim.x * 256) {
    const int m = (int)(i / g.N), n = (int)(i % g.N);
    float v = 0.f;
    for (int z = 0; z < splits; ++z) v += g.part[((size_t)z * g.M + m) * g.ldc + n];
    gemm_epilogue<EPI>(g, m, n, v);
  }
}

// K splits for an M x N x K product: enough blocks to cover the device
// (256 CUs) when the output alone gives too few, each split at least 512 K.
static int gemm_splits(int M, int N, int K) {
  const int blocks = ((N + 63) / 64) * ((M + 63) / 64);
  int sp = 1;
  while (blocks * sp * 2 <= 512 && K / (sp * 2) >= 512) sp *= 2;
  return sp;
}
// Partial-sum floats the split-K path of gemm needs for an M x N product.
static size_t gemm_part_floats(int M, int N, int K) {
  const int sp = gemm_splits(M, N, K);
  return sp > 1 ? (size_t)sp * M * N : 0;
}

__global__ void k_quantize(const float* x, uint16_t* q, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    q[i] = to_bf16(x[i]);
}

// r = y - t; dY = 2 r / (B n_out) (FP32 and BF16); per-block partial sums of r^2.
__global__ __launch_bounds__(256) void k_mse(const float* y, const float* t, size_t n, float scale, float* dy,
                                             uint16_t* dyq, double* part) {
  __shared__ double sh[4];
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float r = y[i] - t[i];
    s += (double)r * (double)r;
    const float d = scale * r;
    dy[i] = d;
    dyq[i] = to_bf16(d);
  }
  s = block_sum_d(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_sum_parts(const double* part, int n, double* out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  s = block_sum_d(s, sh);
  if (threadIdx.x == 0) *out = s;
}

// db[n] = sum over the batch of dz[b][n]: a block takes 64 columns with 16 row
// groups (rows g, g + 16, ...), whose partial sums are added in group order
// through LDS (the same order on every call).
constexpr int kBiasGroups = 16;
__global__ __launch_bounds__(64 * kBiasGroups) void k_bias_grad(const float* dz, int B, int N, float* db) {
  __shared__ float part[kBiasGroups][64];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  float s = 0.f;
  if (n < N) {
#pragma unroll 4
    for (int b = g; b < B; b += kBiasGroups) s += dz[(size_t)b * N + n];
  }
  part[g][c] = s;
  __syncthreads();
  if (g == 0 && n < N) {
    float t = 0.f;
    for (int i = 0; i < kBiasGroups; ++i) t += part[i][c];
    db[n] = t;
  }
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// ---- star warm-start data movement ------------------------------------------
__global__ __launch_bounds__(256) void k_star_features(const StarDesc* st, int L, int n, float shift, float scale,
                                                       float* x) {
  const int i = blockIdx.x / L, l = blockIdx.x % L;
  const double* lg = st[i].lg_leaf + (size_t)l * n;
  float* xo = x + ((size_t)i * L + l) * n;
  for (int p = threadIdx.x; p < n; p += 256) xo[p] = (float)((fmax(lg[p], -40.0) - (double)shift) * (double)scale);
}

__global__ __launch_bounds__(256) void k_star_targets(const StarDesc* st, int L, int n, float out_scale, float* t) {
  __shared__ double sh[4];
  const int i = blockIdx.x / L, l = blockIdx.x % L;
  const double* src = st[i].lam_cur + (size_t)2 * n * l + n;
  double s = 0.0;
  for (int p = threadIdx.x; p < n; p += 256) s += src[p];
  const double mean = block_sum_d(s, sh) / n;
  float* to = t + ((size_t)i * L + l) * n;
  for (int p = threadIdx.x; p < n; p += 256) to[p] = (float)((src[p] - mean) / (double)out_scale);
}

__global__ __launch_bounds__(256) void k_star_apply(const StarDesc* st, int L, int n, const float* y, float out_scale,
                                                    int* rejected) {
  __shared__ double sh[4];
  const int i = blockIdx.x;
  const float* yi = y + (size_t)i * L * n;
  double bad = 0.0;
  for (int p = threadIdx.x; p < L * n; p += 256) bad += isfinite(yi[p]) ? 0.0 : 1.0;
  bad = block_sum_d(bad, sh);
  double* base = st[i].lam0;
  for (int l = 0; l < L; ++l) {
    double s = 0.0;
    if (bad == 0.0)
      for (int p = threadIdx.x; p < n; p += 256) s += yi[(size_t)l * n + p];
    const double mean = block_sum_d(s, sh) / n;
    double* center = base + (size_t)2 * n * l;
    double* leaf = center + n;
    for (int p = threadIdx.x; p < n; p += 256) {
      center[p] = 0.0;
      leaf[p] = bad == 0.0 ? (double)out_scale * ((double)yi[(size_t)l * n + p] - mean) : 0.0;
    }
  }
  if (threadIdx.x == 0 && bad != 0.0) atomicAdd(rejected, 1);
}

hipError_t launch_star_features(const StarDesc* stars, int count, int L, int n, float shift, float scale, float* x,
                                hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_star_features, dim3(count * L), dim3(256), 0, s, stars, L, n, shift, scale, x);
  return hipGetLastError();
}
hipError_t launch_star_targets(const StarDesc* stars, int count, int L, int n, float out_scale, float* t,
                               hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_star_targets, dim3(count * L), dim3(256), 0, s, stars, L, n, out_scale, t);
  return hipGetLastError();
}
hipError_t launch_star_apply(const StarDesc* stars, int count, int L, int n, const float* y, float out_scale,
                             int* rejected, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_star_apply, dim3(count), dim3(256), 0, s, stars, L, n, y, out_scale, rejected);
  return hipGetLastError();
}

}  // namespace gmot

using namespace gmot;

// ---------------------------------------------------------------------------
// MLP host object
// ---------------------------------------------------------------------------
namespace {
thread_local std::string g_mlp_error;
int mfail(int code, const std::string& m) {
  g_mlp_error = m;
  gmot_set_last_error(m);
  return code;
}
#define MCHK(x)                                                                               \
  do {                                                                                        \
    hipError_t e_ = (x);                                                                      \
    if (e_ != hipSuccess) return mfail(GMOT_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
}  // namespace

// ---- workspace of the allocation-free forward pass ---------------------------
// gmot_mlp_forward_static keeps its activations in this file-scope device
// array, so the call needs no allocation; every device the library runs on
// holds its own copy until the process ends.  In host code the array's name is
// a host-side stand-in, not a device address: kernels and copies get the
// address hipGetSymbolAddress returned on the current device (static_ws).
constexpr size_t kStaticWsBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWsBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_ws_mu;
static unsigned char* g_ws_ptr[kMaxDevices] = {};

// With `device` current: the device address of `scratch` on it, looked up on
// the first call for that device and kept.
static int static_ws(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return mfail(GMOT_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_ws_mu);
  if (!g_ws_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return mfail(GMOT_EDEVICE, std::string("static workspace address: ") + hipGetErrorString(e));
    g_ws_ptr[device] = (unsigned char*)p;
  }
  *out = g_ws_ptr[device];
  return GMOT_OK;
}

struct gmot_mlp {
  gmot_ctx* ctx = nullptr;
  unsigned char* static_ws = nullptr;  // device address of `scratch` on ctx->device
  int L = 0;
  std::vector<int> w;
  std::vector<int64_t> offW, offB;
  int64_t nparams = 0;
  void* arena = nullptr;
  float *params = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
  std::vector<uint16_t*> Wq;  // BF16 copies of the weights
  int64_t adam_t = 0;
  // activations for up to `cap` rows
  int cap = 0;
  void* act_arena = nullptr;
  std::vector<float*> H;      // H[0] unused; H[l] = layer l output (FP32), H[L] = y
  std::vector<uint16_t*> Hq;  // Hq[l] = BF16 GEMM input of layer l + 1 (Hq[0] = x)
  std::vector<float*> dZ;     // dZ[l] = gradient wrt pre-activation of layer l
  std::vector<uint16_t*> dZq;
  double* part = nullptr;
  double* loss_dev = nullptr;
  float* split_part = nullptr;  // split-K partial sums of the GEMMs (cap rows)
  float *ws_x = nullptr, *ws_y = nullptr;  // warm-start workspaces (cap rows)

  ~gmot_mlp() {
    if (arena) (void)hipFree(arena);
    if (act_arena) (void)hipFree(act_arena);
  }

  int ensure_cap(int B) {
    if (B <= cap) return GMOT_OK;
    if (act_arena) {
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipFree(act_arena);
      act_arena = nullptr;
    }
    int newcap = std::max(B, 64);
    size_t off = 0;
    auto take = [&](size_t bytes) {
      size_t o = (off + 255) / 256 * 256;
      off = o + std::max<size_t>(bytes, 1);
      return o;
    };
    std::vector<size_t> oH(L + 1), oHq(L + 1), oZ(L + 1), oZq(L + 1);
    for (int l = 0; l <= L; ++l) {
      oH[l] = take(sizeof(float) * (size_t)newcap * w[l]);
      oHq[l] = take(sizeof(uint16_t) * (size_t)newcap * w[l]);
      oZ[l] = take(sizeof(float) * (size_t)newcap * w[l]);
      oZq[l] = take(sizeof(uint16_t) * (size_t)newcap * w[l]);
    }
    const size_t oPart = take(sizeof(double) * 1024);
    const size_t oLoss = take(sizeof(double));
    size_t split_floats = 0;  // forward products (newcap x w[l] x w[l-1]) and input gradients (x w[l])
    for (int l = 1; l <= L; ++l)
      split_floats = std::max({split_floats, gemm_part_floats(newcap, w[l], w[l - 1]),
                               gemm_part_floats(newcap, w[l - 1], w[l])});
    const size_t oSplit = take(sizeof(float) * split_floats);
    const size_t oX = take(sizeof(float) * (size_t)newcap * w[0]);
    const size_t oY = take(sizeof(float) * (size_t)newcap * w[L]);
    if (hipMalloc(&act_arena, off) != hipSuccess) return mfail(GMOT_ENOMEM, "activation buffers");
    char* b = (char*)act_arena;
    H.assign(L + 1, nullptr);
    Hq.assign(L + 1, nullptr);
    dZ.assign(L + 1, nullptr);
    dZq.assign(L + 1, nullptr);
    for (int l = 0; l <= L; ++l) {
      H[l] = (float*)(b + oH[l]);
      Hq[l] = (uint16_t*)(b + oHq[l]);
      dZ[l] = (float*)(b + oZ[l]);
      dZq[l] = (uint16_t*)(b + oZq[l]);
    }
    part = (double*)(b + oPart);
    loss_dev = (double*)(b + oLoss);
    split_part = (float*)(b + oSplit);
    ws_x = (float*)(b + oX);
    ws_y = (float*)(b + oY);
    cap = newcap;
    return GMOT_OK;
  }

  int refresh_wq() {
    for (int l = 1; l <= L; ++l) {
      const size_t n = (size_t)w[l] * w[l - 1];
      hipLaunchKernelGGL(k_quantize, dim3((unsigned)std::min<size_t>(4096, (n + 255) / 256)), dim3(256), 0,
                         ctx->stream, params + offW[l], Wq[l], n);
      MCHK(hipGetLastError());
    }
    return GMOT_OK;
  }
};

// C = A B with the epilogue; with K split, `part` must hold gemm_part_floats
// floats (same splits for the same shape, so results do not depend on the
// caller).
template <bool TA, bool TB, int EPI>
static hipError_t gemm(GemmArgs g, float* part, hipStream_t s) {
  const int sp = gemm_splits(g.M, g.N, g.K);
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, sp);
  if (sp > 1) {
    if (!part || g.ldc != g.N) return hipErrorInvalidValue;
    g.part = part;
    g.k_chunk = ((g.K / sp) + 31) / 32 * 32;
  } else {
    g.part = nullptr;
    g.k_chunk = g.K;
  }
  hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, s, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || sp == 1) return e;
  const size_t total = (size_t)g.M * g.N;
  const unsigned blocks = (unsigned)std::min<size_t>(4096, (total + 255) / 256);
  hipLaunchKernelGGL((k_gemm_reduce<EPI>), dim3(blocks), dim3(256), 0, s, g, sp);
  return hipGetLastError();
}

static int mlp_forward(gmot_mlp* m, const float* x, int B) {
  hipStream_t s = m->ctx->stream;
  const size_t nx = (size_t)B * m->w[0];
  hipLaunchKernelGGL(k_quantize, dim3((unsigned)std::min<size_t>(4096, (nx + 255) / 256)), dim3(256), 0, s, x,
                     m->Hq[0], nx);
  MCHK(hipGetLastError());
  for (int l = 1; l <= m->L; ++l) {
    GemmArgs g{};
    g.A = m->Hq[l - 1];
    g.B = m->Wq[l];
    g.M = B;
    g.N = m->w[l];
    g.K = m->w[l - 1];
    g.lda = m->w[l - 1];
    g.ldb = m->w[l - 1];
    g.ldc = m->w[l];
    g.C = m->H[l];
    g.Cq = l < m->L ? m->Hq[l] : nullptr;
    g.bias = m->params + m->offB[l];
    MCHK((l < m->L ? gemm<false, true, kBiasRelu>(g, m->split_part, s) : gemm<false, true, kBias>(g, m->split_part, s)));
  }
  return GMOT_OK;
}

static int check_batch(gmot_mlp* m, int B) {
  if (B < 8 || (B % 8) != 0) return mfail(GMOT_ENOTSUP, "batch must be a positive multiple of 8");
  return m->ensure_cap(B);
}

extern "C" {

int gmot_mlp_create(gmot_ctx* ctx, int32_t n_layers, const int32_t* widths, uint64_t seed, gmot_mlp** out) {
  if (!ctx || !widths || !out || n_layers < 1) return mfail(GMOT_EINVAL, "bad network description");
  for (int l = 0; l <= n_layers; ++l)
    if (widths[l] < 8 || widths[l] % 8) return mfail(GMOT_ENOTSUP, "layer widths must be multiples of 8");
  MCHK(hipSetDevice(ctx->device));
  std::unique_ptr<gmot_mlp> m(new gmot_mlp());
  m->ctx = ctx;
  {
    const int rc = static_ws(ctx->device, &m->static_ws);
    if (rc) return rc;
  }
  m->L = n_layers;
  m->w.assign(widths, widths + n_layers + 1);
  m->offW.assign(n_layers + 1, 0);
  m->offB.assign(n_layers + 1, 0);
  int64_t o = 0;
  for (int l = 1; l <= n_layers; ++l) {
    m->offW[l] = o;
    o += (int64_t)m->w[l] * m->w[l - 1];
    m->offB[l] = o;
    o += m->w[l];
  }
  m->nparams = o;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t r = (off + 255) / 256 * 256;
    off = r + std::max<size_t>(bytes, 1);
    return r;
  };
  const size_t oP = take(sizeof(float) * o), oG = take(sizeof(float) * o), oM = take(sizeof(float) * o),
               oV = take(sizeof(float) * o);
  std::vector<size_t> oW(n_layers + 1, 0);
  for (int l = 1; l <= n_layers; ++l) oW[l] = take(sizeof(uint16_t) * (size_t)m->w[l] * m->w[l - 1]);
  if (hipMalloc(&m->arena, off) != hipSuccess) return mfail(GMOT_ENOMEM, "parameter buffers");
  char* b = (char*)m->arena;
  m->params = (float*)(b + oP);
  m->grad = (float*)(b + oG);
  m->m1 = (float*)(b + oM);
  m->m2 = (float*)(b + oV);
  m->Wq.assign(n_layers + 1, nullptr);
  for (int l = 1; l <= n_layers; ++l) m->Wq[l] = (uint16_t*)(b + oW[l]);
  // He-uniform weights from a splitmix64 stream, zero biases
  std::vector<float> h(o, 0.f);
  uint64_t st = seed;
  for (int l = 1; l <= n_layers; ++l) {
    const double lim = std::sqrt(6.0 / m->w[l - 1]);
    for (int64_t i = 0; i < (int64_t)m->w[l] * m->w[l - 1]; ++i) {
      const double u = (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
      h[m->offW[l] + i] = (float)((2.0 * u - 1.0) * lim);
    }
  }
  int rc = gmot_mlp_set_params(m.get(), h.data());
  if (rc) return rc;
  gmot_ctx_retain(ctx);
  *out = m.release();
  return GMOT_OK;
}

void gmot_mlp_destroy(gmot_mlp* m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->ctx->stream);
  gmot_ctx* ctx = m->ctx;
  delete m;
  gmot_ctx_release(ctx);
}

int64_t gmot_mlp_num_params(const gmot_mlp* m) { return m ? m->nparams : -1; }

int gmot_mlp_get_params(gmot_mlp* m, float* out) {
  if (!m || !out) return mfail(GMOT_EINVAL, "null network or output");
  MCHK(hipStreamSynchronize(m->ctx->stream));
  MCHK(hipMemcpy(out, m->params, sizeof(float) * m->nparams, hipMemcpyDeviceToHost));
  return GMOT_OK;
}

int gmot_mlp_set_params(gmot_mlp* m, const float* in) {
  if (!m || !in) return mfail(GMOT_EINVAL, "null network or input");
  MCHK(hipStreamSynchronize(m->ctx->stream));
  MCHK(hipMemcpy(m->params, in, sizeof(float) * m->nparams, hipMemcpyHostToDevice));
  MCHK(hipMemsetAsync(m->m1, 0, sizeof(float) * m->nparams, m->ctx->stream));
  MCHK(hipMemsetAsync(m->m2, 0, sizeof(float) * m->nparams, m->ctx->stream));
  m->adam_t = 0;
  return m->refresh_wq();
}

int gmot_mlp_forward_dev(gmot_mlp* m, const float* x_dev, int32_t batch, float* y_dev) {
  if (!m || !x_dev || !y_dev) return mfail(GMOT_EINVAL, "null argument");
  int rc = check_batch(m, batch);
  if (rc) return rc;
  rc = mlp_forward(m, x_dev, batch);
  if (rc) return rc;
  MCHK(hipMemcpyAsync(y_dev, m->H[m->L], sizeof(float) * (size_t)batch * m->w[m->L], hipMemcpyDeviceToDevice,
                      m->ctx->stream));
  return GMOT_OK;
}

// Layout of the static workspace for a batch of B rows: the BF16 copy of x,
// then per hidden layer its FP32 output and BF16 copy (the last layer writes
// y directly).  Returns the bytes used.
static size_t static_layout(const gmot_mlp* m, int64_t B, std::vector<size_t>* oH, std::vector<size_t>* oHq) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t r = (off + 255) / 256 * 256;
    off = r + bytes;
    return r;
  };
  if (oH) oH->assign(m->L + 1, 0);
  if (oHq) oHq->assign(m->L + 1, 0);
  const size_t q0 = take(sizeof(uint16_t) * (size_t)B * m->w[0]);
  if (oHq) (*oHq)[0] = q0;
  for (int l = 1; l < m->L; ++l) {
    const size_t h = take(sizeof(float) * (size_t)B * m->w[l]);
    const size_t q = take(sizeof(uint16_t) * (size_t)B * m->w[l]);
    if (oH) (*oH)[l] = h;
    if (oHq) (*oHq)[l] = q;
  }
  // split-K partial sums of the widest product (the forward GEMMs split like
  // gmot_mlp_forward_dev's, so both give the same bits)
  size_t split_floats = 0;
  for (int l = 1; l <= m->L; ++l) split_floats = std::max(split_floats, gemm_part_floats((int)B, m->w[l], m->w[l - 1]));
  const size_t sp = take(sizeof(float) * split_floats);
  if (oH) (*oH)[0] = sp;  // oH[0] is otherwise unused: the split-K region
  return off;
}

int gmot_mlp_forward_static(gmot_mlp* m, const float* x_dev, int32_t batch, float* y_dev) {
  if (!m || !x_dev || !y_dev) return mfail(GMOT_EINVAL, "null argument");
  if (batch < 8 || (batch % 8) != 0) return mfail(GMOT_ENOTSUP, "batch must be a positive multiple of 8");
  std::vector<size_t> oH, oHq;
  const size_t need = static_layout(m, batch, &oH, &oHq);
  if (need > kStaticWsBytes) {
    int64_t maxB = 0;
    while (static_layout(m, maxB + 8, nullptr, nullptr) <= kStaticWsBytes) maxB += 8;
    return mfail(GMOT_EINVAL, "batch " + std::to_string(batch) + " needs " + std::to_string(need) +
                                  " bytes of the static workspace; it holds " + std::to_string(kStaticWsBytes) +
                                  " (batches of up to " + std::to_string(maxB) + " rows fit for this network)");
  }
  MCHK(hipSetDevice(m->ctx->device));
  hipStream_t s = m->ctx->stream;
  unsigned char* ws = m->static_ws;
  uint16_t* xq = (uint16_t*)(ws + oHq[0]);
  const size_t nx = (size_t)batch * m->w[0];
  hipLaunchKernelGGL(k_quantize, dim3((unsigned)std::min<size_t>(4096, (nx + 255) / 256)), dim3(256), 0, s, x_dev, xq,
                     nx);
  MCHK(hipGetLastError());
  for (int l = 1; l <= m->L; ++l) {
    GemmArgs g{};
    g.A = l == 1 ? xq : (const uint16_t*)(ws + oHq[l - 1]);
    g.B = m->Wq[l];
    g.M = batch;
    g.N = m->w[l];
    g.K = m->w[l - 1];
    g.lda = m->w[l - 1];
    g.ldb = m->w[l - 1];
    g.ldc = m->w[l];
    g.C = l < m->L ? (float*)(ws + oH[l]) : y_dev;
    g.Cq = l < m->L ? (uint16_t*)(ws + oHq[l]) : nullptr;
    g.bias = m->params + m->offB[l];
    float* part = (float*)(ws + oH[0]);
    MCHK((l < m->L ? gemm<false, true, kBiasRelu>(g, part, s) : gemm<false, true, kBias>(g, part, s)));
  }
  return GMOT_OK;
}

int gmot_mlp_loss_grad_dev(gmot_mlp* m, const float* x_dev, const float* t_dev, int32_t batch, double* loss,
                           float* grad_dev) {
  if (!m || !x_dev || !t_dev) return mfail(GMOT_EINVAL, "null argument");
  int rc = check_batch(m, batch);
  if (rc) return rc;
  rc = mlp_forward(m, x_dev, batch);
  if (rc) return rc;
  hipStream_t s = m->ctx->stream;
  const int L = m->L;
  const size_t ny = (size_t)batch * m->w[L];
  const int nblk = (int)std::min<size_t>(1024, (ny + 255) / 256);
  hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(256), 0, s, m->H[L], t_dev, ny, (float)(2.0 / (double)ny), m->dZ[L],
                     m->dZq[L], m->part);
  MCHK(hipGetLastError());
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, m->part, nblk, m->loss_dev);
  MCHK(hipGetLastError());
  for (int l = L; l >= 1; --l) {
    // dW_l = dZ_l^T H_{l-1}: A(m=o, k=b) = dZq[b][o] (transposed), B(k=b, n=i) = Hq[b][i]
    GemmArgs gw{};
    gw.A = m->dZq[l];
    gw.B = m->Hq[l - 1];
    gw.M = m->w[l];
    gw.N = m->w[l - 1];
    gw.K = batch;
    gw.lda = m->w[l];
    gw.ldb = m->w[l - 1];
    gw.ldc = m->w[l - 1];
    gw.C = m->grad + m->offW[l];
    MCHK((gemm<true, false, kStore>(gw, m->split_part, s)));
    hipLaunchKernelGGL(k_bias_grad, dim3((m->w[l] + 63) / 64), dim3(64 * kBiasGroups), 0, s, m->dZ[l], batch,
                       m->w[l], m->grad + m->offB[l]);
    MCHK(hipGetLastError());
    if (l > 1) {
      // dZ_{l-1} = (dZq_l W_l) * (H_{l-1} > 0): A = dZq [b][o], B(k=o, n=i) = Wq[o][i]
      GemmArgs gx{};
      gx.A = m->dZq[l];
      gx.B = m->Wq[l];
      gx.M = batch;
      gx.N = m->w[l - 1];
      gx.K = m->w[l];
      gx.lda = m->w[l];
      gx.ldb = m->w[l - 1];
      gx.ldc = m->w[l - 1];
      gx.C = m->dZ[l - 1];
      gx.Cq = m->dZq[l - 1];
      gx.mask = m->H[l - 1];
      MCHK((gemm<false, false, kMaskRelu>(gx, m->split_part, s)));
    }
  }
  if (grad_dev)
    MCHK(hipMemcpyAsync(grad_dev, m->grad, sizeof(float) * m->nparams, hipMemcpyDeviceToDevice, s));
  if (loss) {
    double sum = 0.0;
    MCHK(hipMemcpyAsync(&sum, m->loss_dev, sizeof(double), hipMemcpyDeviceToHost, s));
    MCHK(hipStreamSynchronize(s));
    *loss = sum / (double)ny;
  }
  return GMOT_OK;
}

int gmot_mlp_adam_step(gmot_mlp* m, float lr, float beta1, float beta2, float adam_eps) {
  if (!m) return mfail(GMOT_EINVAL, "null network");
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(adam_eps > 0.f))
    return mfail(GMOT_EINVAL, "bad Adam hyper-parameters");
  m->adam_t += 1;
  const float c1 = 1.f - std::pow(beta1, (float)m->adam_t);
  const float c2 = 1.f - std::pow(beta2, (float)m->adam_t);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)std::min<int64_t>(4096, (m->nparams + 255) / 256)), dim3(256), 0,
                     m->ctx->stream, m->params, m->grad, m->m1, m->m2, (size_t)m->nparams, lr, beta1, beta2,
                     adam_eps, c1, c2);
  MCHK(hipGetLastError());
  return m->refresh_wq();
}

int gmot_mlp_train_step_dev(gmot_mlp* m, const float* x_dev, const float* t_dev, int32_t batch, float lr,
                            double* loss) {
  int rc = gmot_mlp_loss_grad_dev(m, x_dev, t_dev, batch, loss, nullptr);
  if (rc) return rc;
  return gmot_mlp_adam_step(m, lr, 0.9f, 0.999f, 1e-8f);
}

const char* gmot_mlp_last_error(void) { return g_mlp_error.c_str(); }

}  // extern "C"

// Internal accessors for the runtime's warm-start entry point.
int gmot_mlp_widths(const gmot_mlp* m, int* n_in, int* n_out) {
  *n_in = m->w[0];
  *n_out = m->w[m->L];
  return GMOT_OK;
}
int gmot_mlp_workspace(gmot_mlp* m, int B, float** x, float** y) {
  int rc = m->ensure_cap(B);
  if (rc) return rc;
  *x = m->ws_x;
  *y = m->ws_y;
  return GMOT_OK;
}
