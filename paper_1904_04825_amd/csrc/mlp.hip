// Learned GMRES warm start: a per-element MLP [U, R(U), Y_{i-1}/dt, Y_{i-2}/dt] -> Y_i/dt
// (standardised per field and variable), 2 hidden GELU layers, BF16 operands with
// FP32 accumulation on MFMA, FP32 master weights trained with Adam.
//
// Every matrix product is C[M][N] = A[M][K] B[N][K]^T with both operands stored
// K-contiguous ("NT"); the backward pass gets its transposed operands from the
// epilogues, which write row- and column-major copies where a later product
// needs them.  Each 256-thread workgroup computes a 32 x 32 tile of C, one
// 16 x 16 sub-tile per wavefront, with v_mfma_f32_16x16x16bf16_1k over K.
#include <cmath>

#include "internal.h"

namespace frjf {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4m __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return 0x7FC0;  // NaN
  u += 0x7FFFu + ((u >> 16) & 1u);                                            // nearest, ties to even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

enum { EPI_F32 = 0, EPI_BIAS_GELU = 1, EPI_GELU_GRAD = 2, EPI_BIAS_F32 = 3 };

typedef short bf16x8 __attribute__((ext_vector_type(8)));

// Eight consecutive bf16 of row `row` from column k (zeros past the row's end or past
// nrows): one 16-byte load when aligned and whole, else element by element.
__device__ __forceinline__ bf16x8 load8(const uint16_t* __restrict__ p, int row, int nrows, int k, int K) {
  bf16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
  if (row >= nrows || k >= K) return v;
  const uint16_t* q = p + (size_t)row * K + k;
  if (k + 7 < K && ((((uintptr_t)q) & 15) == 0)) {
    v = *reinterpret_cast<const bf16x8*>(q);
  } else {
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = (k + t < K) ? (short)q[t] : (short)0;
  }
  return v;
}

// C = A B^T (+ bias) with epilogue EPI:
//   EPI_F32:       Cf[m][n] = C
//   EPI_BIAS_F32:  Cf[m][n] = C + bias[n]
//   EPI_BIAS_GELU: z = C + bias -> Z[m][n] (if Z), H[m][n] = bf16(gelu z), Ht[n][m] (if Ht)
//   EPI_GELU_GRAD: d = C * gelu'(Zin[m][n]) -> Cf[m][n] = d (if Cf), H[m][n] = bf16(d), Ht[n][m]
// A workgroup takes a 32 x 32 tile of C (one 16 x 16 sub-tile per wavefront) and the
// K range of split gridDim.z: EPI_F32 with several splits writes its partial tile to
// Cf + z M N (summed by k_sum_splits).  K advances in chunks of 32: every lane loads 16
// bytes of its A row and of its B row (k0 + 8 (lane / 16) .. + 7) and feeds them to two
// v_mfma_f32_16x16x16bf16_1k (the sum over k does not depend on how the k are dealt
// to lanes, as long as A and B agree); KD chunks are loaded ahead of the one in the
// matrix cores.
constexpr int kGemmKD = 4;
template <int EPI>
__global__ void __launch_bounds__(256) k_gemm_nt(const uint16_t* __restrict__ A, const uint16_t* __restrict__ B, int M,
                                                 int N, int K, int kchunks, const float* __restrict__ bias,
                                                 float* __restrict__ Cf, const float* __restrict__ Zin,
                                                 float* __restrict__ Z, uint16_t* __restrict__ H,
                                                 uint16_t* __restrict__ Ht) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 32 + (w >> 1) * 16;
  const int n0 = blockIdx.x * 32 + (w & 1) * 16;
  f32x4m acc = {0.f, 0.f, 0.f, 0.f};
  const int ar = m0 + (lane & 15), bc = n0 + (lane & 15), kq = 8 * (lane >> 4);
  const int kbeg = blockIdx.z * kchunks * 32;
  const int kend = min(K, kbeg + kchunks * 32);
  const int nch = (kend - kbeg + 31) / 32;
  bf16x8 qa[kGemmKD], qb[kGemmKD];
#pragma unroll
  for (int d = 0; d < kGemmKD; ++d) {
    const int k = kbeg + 32 * d + kq;
    qa[d] = d < nch ? load8(A, ar, M, k, kend) : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
    qb[d] = d < nch ? load8(B, bc, N, k, kend) : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
  }
  for (int c = 0; c < nch; c += kGemmKD) {
#pragma unroll
    for (int d = 0; d < kGemmKD; ++d) {
      if (c + d < nch) {
        const bf16x8 a = qa[d], bb = qb[d];
        const int cn = c + d + kGemmKD;
        if (cn < nch) {
          const int k = kbeg + 32 * cn + kq;
          qa[d] = load8(A, ar, M, k, kend);
          qb[d] = load8(B, bc, N, k, kend);
        }
        const bf16x4 a0 = {a[0], a[1], a[2], a[3]}, a1 = {a[4], a[5], a[6], a[7]};
        const bf16x4 b0 = {bb[0], bb[1], bb[2], bb[3]}, b1 = {bb[4], bb[5], bb[6], bb[7]};
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b1, acc, 0, 0, 0);
      }
    }
  }
  const int col = n0 + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = m0 + 4 * (lane >> 4) + r;
    if (row >= M || col >= N) continue;
    const size_t i = (size_t)row * N + col;
    float c = acc[r];
    if constexpr (EPI == EPI_F32) {
      Cf[(size_t)blockIdx.z * M * N + i] = c;
    } else if constexpr (EPI == EPI_BIAS_F32) {
      Cf[i] = c + bias[col];
    } else if constexpr (EPI == EPI_BIAS_GELU) {
      const float z = c + bias[col];
      if (Z != nullptr) Z[i] = z;
      const uint16_t h = f2bf(gelu_f(z));
      H[i] = h;
      if (Ht != nullptr) Ht[(size_t)col * M + row] = h;
    } else {
      const float dv = c * gelu_grad_f(Zin[i]);
      if (Cf != nullptr) Cf[i] = dv;
      const uint16_t d = f2bf(dv);
      H[i] = d;
      if (Ht != nullptr) Ht[(size_t)col * M + row] = d;
    }
  }
}

// out[i] = sum over the splits of part[s n + i], in split order
__global__ void k_sum_splits(const float* __restrict__ part, int S, size_t n, float* __restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    float t = part[i];
    for (int q = 1; q < S; ++q) t += part[(size_t)q * n + i];
    out[i] = t;
  }
}

// Products with a long K (the weight gradients, K = batch) and few output tiles split K
// so that the grid has about 256 workgroups; split partials go to `scratch` (at least
// kMaxSplits M N floats) and are summed in split order.
constexpr int kMaxSplits = 8;
static int gemm_splits(int M, int N, int K) {
  const int tiles = ((M + 31) / 32) * ((N + 31) / 32);
  int sp = 1;
  while (sp < kMaxSplits && tiles * sp * 2 <= 256 && K >= 32 * 8 * sp * 2) sp *= 2;
  return sp;
}

template <int EPI>
static hipError_t gemm(const uint16_t* A, const uint16_t* B, int M, int N, int K, const float* bias, float* Cf,
                       const float* Zin, float* Z, uint16_t* H, uint16_t* Ht, hipStream_t s,
                       float* scratch = nullptr) {
  const int chunks = (K + 31) / 32;
  const int sp = (EPI == EPI_F32 && scratch != nullptr) ? gemm_splits(M, N, K) : 1;
  const int per = (chunks + sp - 1) / sp;
  dim3 grid((N + 31) / 32, (M + 31) / 32, sp);
  float* dst = sp > 1 ? scratch : Cf;
  hipLaunchKernelGGL((k_gemm_nt<EPI>), grid, dim3(256), 0, s, A, B, M, N, K, per, bias, dst, Zin, Z, H, Ht);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || sp == 1) return e;
  const size_t n = (size_t)M * N;
  hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)std::min<size_t>((n + 255) / 256, 1024)), dim3(256), 0, s, scratch,
                     sp, n, Cf);
  return hipGetLastError();
}

// ---------------------------------------------------------------- features
// Row r of X: element elems[r] (or r), feature index f*4*Np + v*Np + k of field f in
// (U, R, Y1/dt, Y2/dt); norm[f][v] = (mean, std).  raw != nullptr: store unnormalised FP32
// into raw[r*stride + ...] (logging); else bf16 standardised into X[r][n_in].
__global__ void k_features(const double* __restrict__ U, const double* __restrict__ R, const double* __restrict__ Y1,
                           const double* __restrict__ Y2, double dt, int nel, int Np, const int* __restrict__ elems,
                           int nrows, const float* __restrict__ norm, uint16_t* __restrict__ X, float* __restrict__ raw,
                           int stride) {
  const int n_in = 16 * Np;
  const size_t total = (size_t)nrows * n_in;
  const double idt = 1.0 / dt;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / n_in), c = (int)(i % n_in);
    const int f = c / (4 * Np), v = (c / Np) % 4, k = c % Np;
    const int e = elems != nullptr ? elems[r] : r;
    const size_t gi = ((size_t)v * nel + e) * Np + k;
    double val;
    if (f == 0) val = U[gi];
    else if (f == 1) val = R[gi];
    else if (f == 2) val = (Y1 != nullptr) ? Y1[gi] * idt : 0.0;
    else val = (Y2 != nullptr) ? Y2[gi] * idt : 0.0;
    if (raw != nullptr) {
      raw[(size_t)r * stride + c] = (float)val;
    } else {
      const float mean = norm[(f * 4 + v) * 2], sd = norm[(f * 4 + v) * 2 + 1];
      X[i] = f2bf((float)((val - mean) / sd));
    }
  }
}

// x0[v][e][k] = (y[e][v*Np + k] * std_v + mean_v) * dt
__global__ void k_decode(const float* __restrict__ y, const float* __restrict__ norm_out, double dt, int nel, int Np,
                         double* __restrict__ x0) {
  const int n_out = 4 * Np;
  const size_t total = (size_t)nel * n_out;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int e = (int)(i / n_out), c = (int)(i % n_out);
    const int v = c / Np, k = c % Np;
    x0[((size_t)v * nel + e) * Np + k] = ((double)y[i] * norm_out[2 * v + 1] + norm_out[2 * v]) * dt;
  }
}

// Logged target: raw[r*stride + n_in + c] = Y[v][e][k] / dt
__global__ void k_log_target(const double* __restrict__ Y, double dt, int nel, int Np, const int* __restrict__ elems,
                             int nrows, float* __restrict__ raw, int stride) {
  const int n_out = 4 * Np, n_in = 16 * Np;
  const size_t total = (size_t)nrows * n_out;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / n_out), c = (int)(i % n_out);
    const int v = c / Np, k = c % Np;
    raw[(size_t)r * stride + n_in + c] = (float)(Y[((size_t)v * nel + elems[r]) * Np + k] / dt);
  }
}

// Mean and deviation of each (field, variable) group over the logged samples: group g < 16
// covers input columns g*Np..; groups 16..19 the target variables.  One workgroup per group.
__global__ void __launch_bounds__(256) k_stats(const float* __restrict__ raw, int count, int stride, int Np,
                                               float* __restrict__ norm) {
  const int g = blockIdx.x;
  const int c0 = (g < 16) ? g * Np : 16 * Np + (g - 16) * Np;
  const size_t n = (size_t)count * Np;
  __shared__ double red[4];
  double s = 0.0;
  for (size_t i = threadIdx.x; i < n; i += 256) s += raw[(i / Np) * stride + c0 + i % Np];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double mean = (red[0] + red[1] + red[2] + red[3]) / (double)n;
  __syncthreads();
  double q = 0.0;
  for (size_t i = threadIdx.x; i < n; i += 256) {
    const double d = raw[(i / Np) * stride + c0 + i % Np] - mean;
    q += d * d;
  }
  for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double sd = sqrt((red[0] + red[1] + red[2] + red[3]) / (double)n);
    const int o = (g < 16) ? 2 * g : 32 + 2 * (g - 16);
    norm[o] = (float)mean;
    norm[o + 1] = (float)(sd > 1e-12 ? sd : 1.0);
  }
}

// Training batch from logged rows idx[]: X bf16 [B][n_in], Xt [n_in][B], T fp32 [B][n_out] (standardised).
__global__ void k_batch(const float* __restrict__ raw, int stride, const int* __restrict__ idx, int B, int Np,
                        const float* __restrict__ norm, uint16_t* __restrict__ X, uint16_t* __restrict__ Xt,
                        float* __restrict__ T) {
  const int n_in = 16 * Np, n_out = 4 * Np, w = n_in + n_out;
  const size_t total = (size_t)B * w;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / w), c = (int)(i % w);
    const float val = raw[(size_t)idx[r] * stride + c];
    if (c < n_in) {
      const int g = c / Np;
      const uint16_t h = f2bf((val - norm[2 * g]) / norm[2 * g + 1]);
      X[(size_t)r * n_in + c] = h;
      Xt[(size_t)c * B + r] = h;
    } else {
      const int v = (c - n_in) / Np;
      T[(size_t)r * n_out + (c - n_in)] = (val - norm[32 + 2 * v]) / norm[32 + 2 * v + 1];
    }
  }
}

// dy = 2 (y - t) / (B n_out): bf16 row- and column-major copies, FP32 copy; loss partials.
__global__ void __launch_bounds__(256) k_mse_grad(const float* __restrict__ Y, const float* __restrict__ T, int B,
                                                  int n_out, uint16_t* __restrict__ dyr, uint16_t* __restrict__ dyt,
                                                  float* __restrict__ dy32, double* __restrict__ partials) {
  const size_t total = (size_t)B * n_out;
  const float sc = 2.0f / (float)total;
  double acc = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const float d = Y[i] - T[i];
    acc += (double)d * d;
    const float g = sc * d;
    dy32[i] = g;
    const uint16_t h = f2bf(g);
    dyr[i] = h;
    dyt[(i % n_out) * B + i / n_out] = h;
  }
  __shared__ double red[4];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// g[n] = sum_m D[m][n] (bf16 or fp32 source).  A workgroup takes 64 columns;
// its 16 row groups each sum every 16th row (coalesced along n), then LDS adds
// the 16 partial sums in a fixed order.
constexpr int kColsumCols = 16, kColsumRows = 64;  // 16 columns per workgroup: enough workgroups for N = 256
__global__ void __launch_bounds__(kColsumCols* kColsumRows)
    k_colsum(const uint16_t* __restrict__ Db, const float* __restrict__ Df, int M, int N, float* __restrict__ g) {
  __shared__ double part[kColsumRows][kColsumCols];
  const int c = threadIdx.x % kColsumCols, r = threadIdx.x / kColsumCols;
  const int n = blockIdx.x * kColsumCols + c;
  double s = 0.0;
  if (n < N) {
    for (int m = r; m < M; m += kColsumRows)
      s += Db != nullptr ? (double)bf2f(Db[(size_t)m * N + n]) : (double)Df[(size_t)m * N + n];
  }
  part[r][c] = s;
  __syncthreads();
  if (r == 0 && n < N) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kColsumRows; ++q) t += part[q][c];
    g[n] = (float)t;
  }
}

// Adam on the FP32 master parameters.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       size_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// bf16 copies W[o][i] and Wt[i][o] of an FP32 matrix
__global__ void k_cast(const float* __restrict__ W, int O, int I, uint16_t* __restrict__ Wb, uint16_t* __restrict__ Wt) {
  const size_t total = (size_t)O * I;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int o = (int)(t / I), i = (int)(t % I);
    const uint16_t h = f2bf(W[t]);
    Wb[t] = h;
    Wt[(size_t)i * O + o] = h;
  }
}

static unsigned grid_for(size_t n) { return (unsigned)std::min<size_t>(std::max<size_t>((n + 255) / 256, 1), 4096); }

// ---------------------------------------------------------------- parameter layout
struct MlpLayout {
  int In, H, Out;
  size_t w1, w2, w3, w1t, w2t, w3t, nw;  // bf16 offsets (elements)
  size_t pW1, pb1, pW2, pb2, pW3, pb3, np;  // fp32 master offsets
};
static MlpLayout layout(int In, int H, int Out) {
  MlpLayout L{};
  L.In = In;
  L.H = H;
  L.Out = Out;
  L.w1 = 0;
  L.w2 = L.w1 + (size_t)H * In;
  L.w3 = L.w2 + (size_t)H * H;
  L.w1t = L.w3 + (size_t)Out * H;
  L.w2t = L.w1t + (size_t)H * In;
  L.w3t = L.w2t + (size_t)H * H;
  L.nw = L.w3t + (size_t)Out * H;
  L.pW1 = 0;
  L.pb1 = L.pW1 + (size_t)H * In;
  L.pW2 = L.pb1 + H;
  L.pb2 = L.pW2 + (size_t)H * H;
  L.pW3 = L.pb2 + H;
  L.pb3 = L.pW3 + (size_t)Out * H;
  L.np = L.pb3 + Out;
  return L;
}

size_t mlp_weight_elems(int In, int H, int Out) { return layout(In, H, Out).nw; }
size_t mlp_param_elems(int In, int H, int Out) { return layout(In, H, Out).np; }

// forward for B rows of X (bf16 [B][In]); Z1/Z2/Ht buffers optional (training)
hipError_t mlp_forward(const fr_mlp* net, const uint16_t* X, int B, float* Y, float* Z1, uint16_t* H1, uint16_t* H1t,
                       float* Z2, uint16_t* H2, uint16_t* H2t, hipStream_t s) {
  const MlpLayout L = layout(net->n_in, net->n_hidden, net->n_out);
  const uint16_t* W = (const uint16_t*)net->d_w;
  const float* b1 = net->d_b;
  const float* b2 = b1 + L.H;
  const float* b3 = b2 + L.H;
  hipError_t e = gemm<EPI_BIAS_GELU>(X, W + L.w1, B, L.H, L.In, b1, nullptr, nullptr, Z1, H1, H1t, s);
  if (e == hipSuccess) e = gemm<EPI_BIAS_GELU>(H1, W + L.w2, B, L.H, L.H, b2, nullptr, nullptr, Z2, H2, H2t, s);
  if (e == hipSuccess) e = gemm<EPI_BIAS_F32>(H2, W + L.w3, B, L.Out, L.H, b3, Y, nullptr, nullptr, nullptr, nullptr, s);
  return e;
}

size_t mlp_infer_bytes(int nel, int In, int H, int Out) {
  return ((size_t)nel * In * 2 + 255) / 256 * 256 + 2 * (((size_t)nel * H * 2 + 255) / 256 * 256) +
         ((size_t)nel * Out * 4 + 255) / 256 * 256;
}

hipError_t mlp_infer(const fr_disc* d, const fr_mlp* net, const double* U, const double* R, const double* Y1,
                     const double* Y2, double dt, double* x0, void* work, hipStream_t s) {
  const int In = net->n_in, H = net->n_hidden, Out = net->n_out, nel = d->nel;
  char* p = (char*)work;
  auto take = [&](size_t b) { void* r = p; p += (b + 255) / 256 * 256; return r; };
  uint16_t* X = (uint16_t*)take((size_t)nel * In * 2);
  uint16_t* H1 = (uint16_t*)take((size_t)nel * H * 2);
  uint16_t* H2 = (uint16_t*)take((size_t)nel * H * 2);
  float* Y = (float*)take((size_t)nel * Out * 4);
  hipLaunchKernelGGL(k_features, dim3(grid_for((size_t)nel * In)), dim3(256), 0, s, U, R, Y1, Y2, dt, nel, d->np,
                     nullptr, nel, net->d_norm, X, nullptr, 0);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = mlp_forward(net, X, nel, Y, nullptr, H1, nullptr, nullptr, H2, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_decode, dim3(grid_for((size_t)nel * Out)), dim3(256), 0, s, Y, net->d_norm + 32, dt, nel, d->np,
                     x0);
  return hipGetLastError();
}

hipError_t mlp_log(const fr_disc* d, fr_stage_log* log, const double* U, const double* R, const double* Y1,
                   const double* Y2, const double* Y, double dt, hipStream_t s) {
  if (log->count + log->per_stage > log->capacity) return hipSuccess;  // full: stop logging
  const int stride = 20 * d->np;
  float* raw = log->d_samples + (size_t)log->count * stride;
  const size_t nin = (size_t)log->per_stage * 16 * d->np;
  hipLaunchKernelGGL(k_features, dim3(grid_for(nin)), dim3(256), 0, s, U, R, Y1, Y2, dt, d->nel, d->np, log->d_elems,
                     log->per_stage, nullptr, nullptr, raw, stride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_log_target, dim3(grid_for((size_t)log->per_stage * 4 * d->np)), dim3(256), 0, s, Y, dt, d->nel,
                     d->np, log->d_elems, log->per_stage, raw, stride);
  e = hipGetLastError();
  if (e == hipSuccess) log->count += log->per_stage;
  return e;
}

hipError_t mlp_stats(const float* raw, int count, int Np, float* norm, hipStream_t s) {
  hipLaunchKernelGGL(k_stats, dim3(20), dim3(256), 0, s, raw, count, 20 * Np, Np, norm);
  return hipGetLastError();
}

size_t mlp_train_bytes(int B, int In, int H, int Out) {
  auto a = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t wmax = (size_t)H * (In > H ? In : H);  // largest weight matrix (split-K partials)
  return 2 * a((size_t)B * In * 2) + 4 * a((size_t)B * H * 4) + 4 * a((size_t)B * H * 2) + a((size_t)B * Out * 4) * 3 +
         2 * a((size_t)B * Out * 2) + 4 * a((size_t)B * H * 2) + a(sizeof(float) * kMaxSplits * wmax) +
         a(sizeof(double) * 4096);
}

hipError_t mlp_train_step(fr_mlp_trainer* tr, const float* raw, const int* idx, int B, int Np, double* loss_partials,
                          int* nparts, void* work, hipStream_t s) {
  fr_mlp* net = &tr->net;
  const int In = net->n_in, H = net->n_hidden, Out = net->n_out;
  const MlpLayout L = layout(In, H, Out);
  char* p = (char*)work;
  auto take = [&](size_t b) { void* r = p; p += (b + 255) / 256 * 256; return r; };
  uint16_t* X = (uint16_t*)take((size_t)B * In * 2);
  uint16_t* Xt = (uint16_t*)take((size_t)B * In * 2);
  float* Z1 = (float*)take((size_t)B * H * 4);
  float* Z2 = (float*)take((size_t)B * H * 4);
  uint16_t* H1 = (uint16_t*)take((size_t)B * H * 2);
  uint16_t* H1t = (uint16_t*)take((size_t)B * H * 2);
  uint16_t* H2 = (uint16_t*)take((size_t)B * H * 2);
  uint16_t* H2t = (uint16_t*)take((size_t)B * H * 2);
  float* Y = (float*)take((size_t)B * Out * 4);
  float* T = (float*)take((size_t)B * Out * 4);
  float* dy32 = (float*)take((size_t)B * Out * 4);
  uint16_t* dyr = (uint16_t*)take((size_t)B * Out * 2);
  uint16_t* dyt = (uint16_t*)take((size_t)B * Out * 2);
  uint16_t* dz2 = (uint16_t*)take((size_t)B * H * 2);
  uint16_t* dz2t = (uint16_t*)take((size_t)B * H * 2);
  uint16_t* dz1 = (uint16_t*)take((size_t)B * H * 2);
  uint16_t* dz1t = (uint16_t*)take((size_t)B * H * 2);
  float* dz2f = (float*)take((size_t)B * H * 4);  // hidden gradients before the bf16 rounding (bias sums)
  float* dz1f = (float*)take((size_t)B * H * 4);
  float* gsplit = (float*)take(sizeof(float) * kMaxSplits * (size_t)H * (In > H ? In : H));
  const uint16_t* W = (const uint16_t*)net->d_w;
  float* g = tr->d_grad;
  hipLaunchKernelGGL(k_batch, dim3(grid_for((size_t)B * (In + Out))), dim3(256), 0, s, raw, 20 * Np, idx, B, Np,
                     net->d_norm, X, Xt, T);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = mlp_forward(net, X, B, Y, Z1, H1, H1t, Z2, H2, H2t, s);
  if (e != hipSuccess) return e;
  const unsigned gb = std::min<unsigned>(grid_for((size_t)B * Out), 1024);
  hipLaunchKernelGGL(k_mse_grad, dim3(gb), dim3(256), 0, s, Y, T, B, Out, dyr, dyt, dy32, loss_partials);
  *nparts = (int)gb;
  e = hipGetLastError();
  // weight and bias gradients, layer by layer
  if (e == hipSuccess) e = gemm<EPI_F32>(dyt, H2t, Out, H, B, nullptr, g + L.pW3, nullptr, nullptr, nullptr, nullptr, s, gsplit);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_colsum, dim3((Out + kColsumCols - 1) / kColsumCols), dim3(kColsumCols * kColsumRows), 0, s, nullptr, dy32, B, Out, g + L.pb3);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = gemm<EPI_GELU_GRAD>(dyr, W + L.w3t, B, H, Out, nullptr, dz2f, Z2, nullptr, dz2, dz2t, s);
  if (e == hipSuccess) e = gemm<EPI_F32>(dz2t, H1t, H, H, B, nullptr, g + L.pW2, nullptr, nullptr, nullptr, nullptr, s, gsplit);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_colsum, dim3((H + kColsumCols - 1) / kColsumCols), dim3(kColsumCols * kColsumRows), 0, s, nullptr, dz2f, B, H, g + L.pb2);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = gemm<EPI_GELU_GRAD>(dz2, W + L.w2t, B, H, H, nullptr, dz1f, Z1, nullptr, dz1, dz1t, s);
  if (e == hipSuccess) e = gemm<EPI_F32>(dz1t, Xt, H, In, B, nullptr, g + L.pW1, nullptr, nullptr, nullptr, nullptr, s, gsplit);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_colsum, dim3((H + kColsumCols - 1) / kColsumCols), dim3(kColsumCols * kColsumRows), 0, s, nullptr, dz1f, B, H, g + L.pb1);
    e = hipGetLastError();
  }
  if (e != hipSuccess || tr->lr <= 0.0f) return e;  // lr <= 0: gradients only
  tr->t += 1;
  const float c1 = 1.0f - powf(tr->beta1, (float)tr->t), c2 = 1.0f - powf(tr->beta2, (float)tr->t);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(L.np)), dim3(256), 0, s, tr->d_master, g, tr->d_m, tr->d_v, L.np, tr->lr,
                     tr->beta1, tr->beta2, tr->eps, c1, c2);
  e = hipGetLastError();
  if (e == hipSuccess) e = mlp_sync_weights(tr, s);
  return e;
}

// bf16 weights and fp32 biases of the network from the FP32 master copy
hipError_t mlp_sync_weights(fr_mlp_trainer* tr, hipStream_t s) {
  fr_mlp* net = &tr->net;
  const MlpLayout L = layout(net->n_in, net->n_hidden, net->n_out);
  uint16_t* W = (uint16_t*)net->d_w;
  const float* m = tr->d_master;
  hipLaunchKernelGGL(k_cast, dim3(grid_for((size_t)L.H * L.In)), dim3(256), 0, s, m + L.pW1, L.H, L.In, W + L.w1,
                     W + L.w1t);
  hipLaunchKernelGGL(k_cast, dim3(grid_for((size_t)L.H * L.H)), dim3(256), 0, s, m + L.pW2, L.H, L.H, W + L.w2,
                     W + L.w2t);
  hipLaunchKernelGGL(k_cast, dim3(grid_for((size_t)L.Out * L.H)), dim3(256), 0, s, m + L.pW3, L.Out, L.H, W + L.w3,
                     W + L.w3t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  float* b = (float*)net->d_b;
  e = hipMemcpyAsync(b, m + L.pb1, sizeof(float) * L.H, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(b + L.H, m + L.pb2, sizeof(float) * L.H, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(b + 2 * L.H, m + L.pb3, sizeof(float) * L.Out, hipMemcpyDeviceToDevice, s);
  return e;
}

}  // namespace frjf
