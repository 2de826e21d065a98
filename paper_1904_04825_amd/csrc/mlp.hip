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
#include <vector>

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
// Up to kMaxGroup networks of equal sizes share a launch (the stage networks trained
// together): blockIdx.z = net * splits + split, and every operand is a per-network
// pointer.  A workgroup takes a 32 x 32 tile of C (one 16 x 16 sub-tile per wavefront)
// and the K range of its split: EPI_F32 with several splits writes its partial tile to
// Cf + split M N (summed by k_sum_splits).  K advances in chunks of 32: every lane loads
// 16 bytes of its A row and of its B row (k0 + 8 (lane / 16) .. + 7) and feeds them to
// two v_mfma_f32_16x16x16bf16_1k (the sum over k does not depend on how the k are dealt
// to lanes, as long as A and B agree); KD chunks are loaded ahead of the one in the
// matrix cores.
constexpr int kMaxGroup = kMlpGroupMax;
template <typename T>
struct PerNet {
  T p[kMaxGroup];
};
template <typename T>
static PerNet<T> one(T v) {
  PerNet<T> r{};
  r.p[0] = v;
  return r;
}
struct GemmOps {
  PerNet<const uint16_t*> A, B;
  PerNet<const float*> bias, Zin;
  PerNet<float*> Cf, Z;
  PerNet<uint16_t*> H, Ht;
};

constexpr int kGemmKD = 4;
template <int EPI>
__global__ void __launch_bounds__(256) k_gemm_nt(GemmOps ops, int M, int N, int K, int kchunks, int splits) {
  const int net = blockIdx.z / splits, split = blockIdx.z - net * splits;
  const uint16_t* __restrict__ A = ops.A.p[net];
  const uint16_t* __restrict__ B = ops.B.p[net];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 32 + (w >> 1) * 16;
  const int n0 = blockIdx.x * 32 + (w & 1) * 16;
  f32x4m acc = {0.f, 0.f, 0.f, 0.f};
  const int ar = m0 + (lane & 15), bc = n0 + (lane & 15), kq = 8 * (lane >> 4);
  const int kbeg = split * kchunks * 32;
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
  float* __restrict__ Cf = ops.Cf.p[net];
  const int col = n0 + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = m0 + 4 * (lane >> 4) + r;
    if (row >= M || col >= N) continue;
    const size_t i = (size_t)row * N + col;
    float c = acc[r];
    if constexpr (EPI == EPI_F32) {
      Cf[(size_t)split * M * N + i] = c;
    } else if constexpr (EPI == EPI_BIAS_F32) {
      Cf[i] = c + ops.bias.p[net][col];
    } else if constexpr (EPI == EPI_BIAS_GELU) {
      const float z = c + ops.bias.p[net][col];
      if (ops.Z.p[net] != nullptr) ops.Z.p[net][i] = z;
      const uint16_t h = f2bf(gelu_f(z));
      ops.H.p[net][i] = h;
      if (ops.Ht.p[net] != nullptr) ops.Ht.p[net][(size_t)col * M + row] = h;
    } else {
      const float dv = c * gelu_grad_f(ops.Zin.p[net][i]);
      if (Cf != nullptr) Cf[i] = dv;
      const uint16_t d = f2bf(dv);
      ops.H.p[net][i] = d;
      if (ops.Ht.p[net] != nullptr) ops.Ht.p[net][(size_t)col * M + row] = d;
    }
  }
}

// out[i] = sum over the splits of part[s n + i], in split order (network blockIdx.y)
__global__ void k_sum_splits(PerNet<float*> part, int S, size_t n, PerNet<float*> out) {
  const float* __restrict__ pp = part.p[blockIdx.y];
  float* __restrict__ o = out.p[blockIdx.y];
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    float t = pp[i];
    for (int q = 1; q < S; ++q) t += pp[(size_t)q * n + i];
    o[i] = t;
  }
}

// Products with a long K (the weight gradients, K = batch) and few output tiles split K
// so that one network's grid has about 256 workgroups; split partials go to `scratch`
// (per network, at least kMaxSplits M N floats) and are summed in split order.  The
// split count depends on the product's shape only, so a network's result does not
// depend on how many networks share the launch.
constexpr int kMaxSplits = 8;
static int gemm_splits(int M, int N, int K) {
  const int tiles = ((M + 31) / 32) * ((N + 31) / 32);
  int sp = 1;
  while (sp < kMaxSplits && tiles * sp * 2 <= 256 && K >= 32 * 8 * sp * 2) sp *= 2;
  return sp;
}

template <int EPI>
static hipError_t gemm(GemmOps ops, int count, int M, int N, int K, hipStream_t s,
                       const PerNet<float*>* scratch = nullptr) {
  const int chunks = (K + 31) / 32;
  const int sp = (EPI == EPI_F32 && scratch != nullptr) ? gemm_splits(M, N, K) : 1;
  const int per = (chunks + sp - 1) / sp;
  const PerNet<float*> dst = ops.Cf;
  if (sp > 1) ops.Cf = *scratch;
  dim3 grid((N + 31) / 32, (M + 31) / 32, sp * count);
  hipLaunchKernelGGL((k_gemm_nt<EPI>), grid, dim3(256), 0, s, ops, M, N, K, per, sp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || sp == 1) return e;
  const size_t n = (size_t)M * N;
  hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)std::min<size_t>((n + 255) / 256, 1024), count), dim3(256), 0, s,
                     *scratch, sp, n, dst);
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

// Training batch from logged rows idx[]: X bf16 [B][n_in], Xt [n_in][B], T fp32 [B][n_out]
// (standardised); network blockIdx.y.
__global__ void k_batch(PerNet<const float*> rawn, int stride, PerNet<const int*> idxn, int B, int Np,
                        PerNet<const float*> normn, PerNet<uint16_t*> Xn, PerNet<uint16_t*> Xtn, PerNet<float*> Tn) {
  const float* __restrict__ raw = rawn.p[blockIdx.y];
  const int* __restrict__ idx = idxn.p[blockIdx.y];
  const float* __restrict__ norm = normn.p[blockIdx.y];
  uint16_t* __restrict__ X = Xn.p[blockIdx.y];
  uint16_t* __restrict__ Xt = Xtn.p[blockIdx.y];
  float* __restrict__ T = Tn.p[blockIdx.y];
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

// dy = 2 (y - t) / (B n_out): bf16 row- and column-major copies, FP32 copy; loss
// partials (one per workgroup); network blockIdx.y.
__global__ void __launch_bounds__(256) k_mse_grad(PerNet<const float*> Yn, PerNet<const float*> Tn, int B, int n_out,
                                                  PerNet<uint16_t*> dyrn, PerNet<uint16_t*> dytn,
                                                  PerNet<float*> dy32n, PerNet<double*> partn) {
  const float* __restrict__ Y = Yn.p[blockIdx.y];
  const float* __restrict__ T = Tn.p[blockIdx.y];
  uint16_t* __restrict__ dyr = dyrn.p[blockIdx.y];
  uint16_t* __restrict__ dyt = dytn.p[blockIdx.y];
  float* __restrict__ dy32 = dy32n.p[blockIdx.y];
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
  if (threadIdx.x == 0) partn.p[blockIdx.y][blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// g[n] = sum_m D[m][n] (the bias gradients, from the FP32 output gradients before their
// bf16 rounding).  A workgroup takes 16 columns; its 64 row groups each sum every 64th
// row (coalesced along n), then LDS adds the 64 partial sums in a fixed order.
// Network blockIdx.y.
constexpr int kColsumCols = 16, kColsumRows = 64;  // 16 columns per workgroup: enough workgroups for N = 256
__global__ void __launch_bounds__(kColsumCols* kColsumRows)
    k_colsum(PerNet<const float*> Dn, int M, int N, PerNet<float*> gn) {
  const float* __restrict__ Df = Dn.p[blockIdx.y];
  __shared__ double part[kColsumRows][kColsumCols];
  const int c = threadIdx.x % kColsumCols, r = threadIdx.x / kColsumCols;
  const int n = blockIdx.x * kColsumCols + c;
  double s = 0.0;
  if (n < N) {
    for (int m = r; m < M; m += kColsumRows) s += (double)Df[(size_t)m * N + n];
  }
  part[r][c] = s;
  __syncthreads();
  if (r == 0 && n < N) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kColsumRows; ++q) t += part[q][c];
    gn.p[blockIdx.y][n] = (float)t;
  }
}

// Adam on the FP32 master parameters of network blockIdx.y (skipped when its lr <= 0).
struct AdamCoef {
  float lr, b1, b2, eps, c1, c2;
};
__global__ void k_adam(PerNet<float*> pn, PerNet<const float*> gn, PerNet<float*> mn, PerNet<float*> vn, size_t n,
                       PerNet<AdamCoef> cn) {
  const AdamCoef co = cn.p[blockIdx.y];
  if (!(co.lr > 0.0f)) return;
  float* __restrict__ p = pn.p[blockIdx.y];
  const float* __restrict__ g = gn.p[blockIdx.y];
  float* __restrict__ m = mn.p[blockIdx.y];
  float* __restrict__ v = vn.p[blockIdx.y];
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = co.b1 * m[i] + (1.0f - co.b1) * gi;
    const float vi = co.b2 * v[i] + (1.0f - co.b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= co.lr * (mi / co.c1) / (sqrtf(vi / co.c2) + co.eps);
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

// bf16 weights (row-major W[o][i] and transposed Wt[i][o] copies of W1, W2, W3) and FP32
// biases of network blockIdx.y from its master copy; networks with on == 0 are left alone.
__global__ void k_sync(PerNet<const float*> mastern, PerNet<uint16_t*> Wn, PerNet<float*> bn, PerNet<int> on,
                       MlpLayout L) {
  if (!on.p[blockIdx.y]) return;
  const float* __restrict__ m = mastern.p[blockIdx.y];
  uint16_t* __restrict__ W = Wn.p[blockIdx.y];
  float* __restrict__ b = bn.p[blockIdx.y];
  const size_t n1 = (size_t)L.H * L.In, n2 = (size_t)L.H * L.H, n3 = (size_t)L.Out * L.H;
  const size_t total = n1 + n2 + n3 + 2 * (size_t)L.H + L.Out;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    if (t < n1) {
      const uint16_t h = f2bf(m[L.pW1 + t]);
      W[L.w1 + t] = h;
      W[L.w1t + (t % L.In) * L.H + t / L.In] = h;
    } else if (t < n1 + n2) {
      const size_t u = t - n1;
      const uint16_t h = f2bf(m[L.pW2 + u]);
      W[L.w2 + u] = h;
      W[L.w2t + (u % L.H) * L.H + u / L.H] = h;
    } else if (t < n1 + n2 + n3) {
      const size_t u = t - n1 - n2;
      const uint16_t h = f2bf(m[L.pW3 + u]);
      W[L.w3 + u] = h;
      W[L.w3t + (u % L.H) * L.Out + u / L.H] = h;
    } else {
      const size_t u = t - n1 - n2 - n3;  // b1 | b2 | b3
      const size_t src = u < (size_t)L.H ? L.pb1 + u : (u < 2 * (size_t)L.H ? L.pb2 + u - L.H : L.pb3 + u - 2 * L.H);
      b[u] = m[src];
    }
  }
}

size_t mlp_weight_elems(int In, int H, int Out) { return layout(In, H, Out).nw; }
size_t mlp_param_elems(int In, int H, int Out) { return layout(In, H, Out).np; }

// forward for B rows of X (bf16 [B][In]) of one network
hipError_t mlp_forward(const fr_mlp* net, const uint16_t* X, int B, float* Y, uint16_t* H1, uint16_t* H2,
                       hipStream_t s) {
  const MlpLayout L = layout(net->n_in, net->n_hidden, net->n_out);
  const uint16_t* W = (const uint16_t*)net->d_w;
  const float* b1 = net->d_b;
  GemmOps o{};
  o.A = one<const uint16_t*>(X);
  o.B = one<const uint16_t*>(W + L.w1);
  o.bias = one<const float*>(b1);
  o.H = one(H1);
  hipError_t e = gemm<EPI_BIAS_GELU>(o, 1, B, L.H, L.In, s);
  o.A = one<const uint16_t*>(H1);
  o.B = one<const uint16_t*>(W + L.w2);
  o.bias = one<const float*>(b1 + L.H);
  o.H = one(H2);
  if (e == hipSuccess) e = gemm<EPI_BIAS_GELU>(o, 1, B, L.H, L.H, s);
  o = GemmOps{};
  o.A = one<const uint16_t*>(H2);
  o.B = one<const uint16_t*>(W + L.w3);
  o.bias = one<const float*>(b1 + 2 * L.H);
  o.Cf = one(Y);
  if (e == hipSuccess) e = gemm<EPI_BIAS_F32>(o, 1, B, L.Out, L.H, s);
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
  if (e == hipSuccess) e = mlp_forward(net, X, nel, Y, H1, H2, s);
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

constexpr int kLossParts = 1024;  // loss partials per network and step (k_mse_grad workgroups)

size_t mlp_train_bytes(int B, int In, int H, int Out) {
  auto a = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t wmax = (size_t)H * (In > H ? In : H);  // largest weight matrix (split-K partials)
  return 2 * a((size_t)B * In * 2) + 4 * a((size_t)B * H * 4) + 4 * a((size_t)B * H * 2) + a((size_t)B * Out * 4) * 3 +
         2 * a((size_t)B * Out * 2) + 4 * a((size_t)B * H * 2) + a(sizeof(float) * kMaxSplits * wmax) +
         a(sizeof(double) * kLossParts);
}

// One network's training buffers, carved from its mlp_train_bytes workspace (the loss
// partials last).
struct TrainBufs {
  uint16_t *X, *Xt;
  float *Z1, *Z2;
  uint16_t *H1, *H1t, *H2, *H2t;
  float *Y, *T, *dy32;
  uint16_t *dyr, *dyt, *dz2, *dz2t, *dz1, *dz1t;
  float *dz2f, *dz1f;  // hidden gradients before the bf16 rounding (bias sums)
  float* gsplit;
  double* partials;
};
static TrainBufs carve(void* work, int B, int In, int H, int Out) {
  char* p = (char*)work;
  auto take = [&](size_t b) { void* r = p; p += (b + 255) / 256 * 256; return r; };
  TrainBufs t;
  t.X = (uint16_t*)take((size_t)B * In * 2);
  t.Xt = (uint16_t*)take((size_t)B * In * 2);
  t.Z1 = (float*)take((size_t)B * H * 4);
  t.Z2 = (float*)take((size_t)B * H * 4);
  t.H1 = (uint16_t*)take((size_t)B * H * 2);
  t.H1t = (uint16_t*)take((size_t)B * H * 2);
  t.H2 = (uint16_t*)take((size_t)B * H * 2);
  t.H2t = (uint16_t*)take((size_t)B * H * 2);
  t.Y = (float*)take((size_t)B * Out * 4);
  t.T = (float*)take((size_t)B * Out * 4);
  t.dy32 = (float*)take((size_t)B * Out * 4);
  t.dyr = (uint16_t*)take((size_t)B * Out * 2);
  t.dyt = (uint16_t*)take((size_t)B * Out * 2);
  t.dz2 = (uint16_t*)take((size_t)B * H * 2);
  t.dz2t = (uint16_t*)take((size_t)B * H * 2);
  t.dz1 = (uint16_t*)take((size_t)B * H * 2);
  t.dz1t = (uint16_t*)take((size_t)B * H * 2);
  t.dz2f = (float*)take((size_t)B * H * 4);
  t.dz1f = (float*)take((size_t)B * H * 4);
  t.gsplit = (float*)take(sizeof(float) * kMaxSplits * (size_t)H * (In > H ? In : H));
  t.partials = (double*)take(sizeof(double) * kLossParts);
  return t;
}

template <typename T, typename F>
static PerNet<T> per_net(int count, F f) {
  PerNet<T> r{};
  for (int q = 0; q < count; ++q) r.p[q] = f(q);
  return r;
}

// Weights and biases of each network from its master copy (networks with on[q] == 0 skipped).
static hipError_t sync_group(fr_mlp_trainer* const* trs, int count, const int* on, hipStream_t s) {
  const fr_mlp& n0 = trs[0]->net;
  const MlpLayout L = layout(n0.n_in, n0.n_hidden, n0.n_out);
  const size_t total = L.nw / 2 + 2 * (size_t)L.H + L.Out;
  hipLaunchKernelGGL(k_sync, dim3(grid_for(total), count), dim3(256), 0, s,
                     per_net<const float*>(count, [&](int q) { return (const float*)trs[q]->d_master; }),
                     per_net<uint16_t*>(count, [&](int q) { return (uint16_t*)trs[q]->net.d_w; }),
                     per_net<float*>(count, [&](int q) { return trs[q]->net.d_b; }),
                     per_net<int>(count, [&](int q) { return on == nullptr ? 1 : on[q]; }), L);
  return hipGetLastError();
}

hipError_t mlp_sync_weights(fr_mlp_trainer* tr, hipStream_t s) { return sync_group(&tr, 1, nullptr, s); }

// One training step of `count` networks of equal sizes, each on its own logged rows:
// network q reads raws[q] rows idx[q][0..B) and uses the workspace works[q]
// (mlp_train_bytes).  Every kernel is launched once for all networks; network q's
// arithmetic is the same whatever count is.
hipError_t mlp_train_group(fr_mlp_trainer* const* trs, const float* const* raws, const int* const* idx, int count,
                           int B, int Np, void* const* works, int* nparts, hipStream_t s) {
  const fr_mlp& n0 = trs[0]->net;
  const int In = n0.n_in, H = n0.n_hidden, Out = n0.n_out;
  const MlpLayout L = layout(In, H, Out);
  TrainBufs tb[kMaxGroup];
  for (int q = 0; q < count; ++q) tb[q] = carve(works[q], B, In, H, Out);
  auto W = [&](int q) { return (const uint16_t*)trs[q]->net.d_w; };
  auto G = [&](int q) { return trs[q]->d_grad; };
  auto gs = per_net<float*>(count, [&](int q) { return tb[q].gsplit; });
  hipLaunchKernelGGL(k_batch, dim3(grid_for((size_t)B * (In + Out)), count), dim3(256), 0, s,
                     per_net<const float*>(count, [&](int q) { return raws[q]; }), 20 * Np,
                     per_net<const int*>(count, [&](int q) { return idx[q]; }), B, Np,
                     per_net<const float*>(count, [&](int q) { return (const float*)trs[q]->net.d_norm; }),
                     per_net<uint16_t*>(count, [&](int q) { return tb[q].X; }),
                     per_net<uint16_t*>(count, [&](int q) { return tb[q].Xt; }),
                     per_net<float*>(count, [&](int q) { return tb[q].T; }));
  hipError_t e = hipGetLastError();
  // forward, keeping Z1, Z2 and the transposed activations for the backward products
  GemmOps o{};
  o.A = per_net<const uint16_t*>(count, [&](int q) { return tb[q].X; });
  o.B = per_net<const uint16_t*>(count, [&](int q) { return W(q) + L.w1; });
  o.bias = per_net<const float*>(count, [&](int q) { return (const float*)trs[q]->net.d_b; });
  o.Z = per_net<float*>(count, [&](int q) { return tb[q].Z1; });
  o.H = per_net<uint16_t*>(count, [&](int q) { return tb[q].H1; });
  o.Ht = per_net<uint16_t*>(count, [&](int q) { return tb[q].H1t; });
  if (e == hipSuccess) e = gemm<EPI_BIAS_GELU>(o, count, B, H, In, s);
  o.A = per_net<const uint16_t*>(count, [&](int q) { return tb[q].H1; });
  o.B = per_net<const uint16_t*>(count, [&](int q) { return W(q) + L.w2; });
  o.bias = per_net<const float*>(count, [&](int q) { return (const float*)trs[q]->net.d_b + H; });
  o.Z = per_net<float*>(count, [&](int q) { return tb[q].Z2; });
  o.H = per_net<uint16_t*>(count, [&](int q) { return tb[q].H2; });
  o.Ht = per_net<uint16_t*>(count, [&](int q) { return tb[q].H2t; });
  if (e == hipSuccess) e = gemm<EPI_BIAS_GELU>(o, count, B, H, H, s);
  o = GemmOps{};
  o.A = per_net<const uint16_t*>(count, [&](int q) { return tb[q].H2; });
  o.B = per_net<const uint16_t*>(count, [&](int q) { return W(q) + L.w3; });
  o.bias = per_net<const float*>(count, [&](int q) { return (const float*)trs[q]->net.d_b + 2 * H; });
  o.Cf = per_net<float*>(count, [&](int q) { return tb[q].Y; });
  if (e == hipSuccess) e = gemm<EPI_BIAS_F32>(o, count, B, Out, H, s);
  if (e != hipSuccess) return e;
  const unsigned gb = std::min<unsigned>(grid_for((size_t)B * Out), kLossParts);
  hipLaunchKernelGGL(k_mse_grad, dim3(gb, count), dim3(256), 0, s,
                     per_net<const float*>(count, [&](int q) { return (const float*)tb[q].Y; }),
                     per_net<const float*>(count, [&](int q) { return (const float*)tb[q].T; }), B, Out,
                     per_net<uint16_t*>(count, [&](int q) { return tb[q].dyr; }),
                     per_net<uint16_t*>(count, [&](int q) { return tb[q].dyt; }),
                     per_net<float*>(count, [&](int q) { return tb[q].dy32; }),
                     per_net<double*>(count, [&](int q) { return tb[q].partials; }));
  *nparts = (int)gb;
  e = hipGetLastError();
  // weight and bias gradients, layer by layer
  auto wgrad = [&](auto A, auto Bm, int M, int N, size_t off) {
    GemmOps g{};
    g.A = per_net<const uint16_t*>(count, A);
    g.B = per_net<const uint16_t*>(count, Bm);
    g.Cf = per_net<float*>(count, [&](int q) { return G(q) + off; });
    return gemm<EPI_F32>(g, count, M, N, B, s, &gs);
  };
  auto bgrad = [&](auto D, int N, size_t off) {
    hipLaunchKernelGGL(k_colsum, dim3((N + kColsumCols - 1) / kColsumCols, count), dim3(kColsumCols * kColsumRows), 0,
                       s, per_net<const float*>(count, D), B, N,
                       per_net<float*>(count, [&](int q) { return G(q) + off; }));
    return hipGetLastError();
  };
  auto hgrad = [&](auto A, auto Bm, int N, int K, auto Zin, auto Cf, auto Hh, auto Ht) {
    GemmOps g{};
    g.A = per_net<const uint16_t*>(count, A);
    g.B = per_net<const uint16_t*>(count, Bm);
    g.Zin = per_net<const float*>(count, Zin);
    g.Cf = per_net<float*>(count, Cf);
    g.H = per_net<uint16_t*>(count, Hh);
    g.Ht = per_net<uint16_t*>(count, Ht);
    return gemm<EPI_GELU_GRAD>(g, count, B, N, K, s);
  };
  if (e == hipSuccess)
    e = wgrad([&](int q) { return tb[q].dyt; }, [&](int q) { return tb[q].H2t; }, Out, H, L.pW3);
  if (e == hipSuccess) e = bgrad([&](int q) { return tb[q].dy32; }, Out, L.pb3);
  if (e == hipSuccess)
    e = hgrad([&](int q) { return tb[q].dyr; }, [&](int q) { return W(q) + L.w3t; }, H, Out,
              [&](int q) { return tb[q].Z2; }, [&](int q) { return tb[q].dz2f; }, [&](int q) { return tb[q].dz2; },
              [&](int q) { return tb[q].dz2t; });
  if (e == hipSuccess)
    e = wgrad([&](int q) { return tb[q].dz2t; }, [&](int q) { return tb[q].H1t; }, H, H, L.pW2);
  if (e == hipSuccess) e = bgrad([&](int q) { return tb[q].dz2f; }, H, L.pb2);
  if (e == hipSuccess)
    e = hgrad([&](int q) { return tb[q].dz2; }, [&](int q) { return W(q) + L.w2t; }, H, H,
              [&](int q) { return tb[q].Z1; }, [&](int q) { return tb[q].dz1f; }, [&](int q) { return tb[q].dz1; },
              [&](int q) { return tb[q].dz1t; });
  if (e == hipSuccess)
    e = wgrad([&](int q) { return tb[q].dz1t; }, [&](int q) { return tb[q].Xt; }, H, In, L.pW1);
  if (e == hipSuccess) e = bgrad([&](int q) { return tb[q].dz1f; }, H, L.pb1);
  if (e != hipSuccess) return e;
  // Adam (networks with lr <= 0 keep gradients only), then the bf16 weights
  int on[kMaxGroup] = {0};
  bool any = false;
  PerNet<AdamCoef> co{};
  for (int q = 0; q < count; ++q) {
    fr_mlp_trainer* tr = trs[q];
    if (!(tr->lr > 0.0f)) continue;
    tr->t += 1;
    co.p[q] = AdamCoef{tr->lr, tr->beta1, tr->beta2, tr->eps, 1.0f - powf(tr->beta1, (float)tr->t),
                       1.0f - powf(tr->beta2, (float)tr->t)};
    on[q] = 1;
    any = true;
  }
  if (!any) return hipSuccess;
  hipLaunchKernelGGL(k_adam, dim3(grid_for(L.np), count), dim3(256), 0, s,
                     per_net<float*>(count, [&](int q) { return trs[q]->d_master; }),
                     per_net<const float*>(count, [&](int q) { return (const float*)trs[q]->d_grad; }),
                     per_net<float*>(count, [&](int q) { return trs[q]->d_m; }),
                     per_net<float*>(count, [&](int q) { return trs[q]->d_v; }), L.np, co);
  e = hipGetLastError();
  if (e == hipSuccess) e = sync_group(trs, count, on, s);
  return e;
}

// Batch MSE of the last step of each network: the loss partials of works[q] summed on the host.
hipError_t mlp_group_loss(void* const* works, int count, int B, int In, int H, int Out, int nparts, double* h_loss,
                          hipStream_t s) {
  std::vector<double> h((size_t)count * nparts);
  for (int q = 0; q < count; ++q) {
    const TrainBufs t = carve(works[q], B, In, H, Out);
    hipError_t e = hipMemcpyAsync(h.data() + (size_t)q * nparts, t.partials, sizeof(double) * nparts,
                                  hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  for (int q = 0; q < count; ++q) {
    double sum = 0.0;
    for (int i = 0; i < nparts; ++i) sum += h[(size_t)q * nparts + i];
    h_loss[q] = sum / ((double)B * Out);
  }
  return hipSuccess;
}

}  // namespace frjf
