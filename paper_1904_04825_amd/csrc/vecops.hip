// Vector kernels of the GMRES layer (Section 4.5): deterministic norms,
// linear combinations, classical Gram-Schmidt with one re-orthogonalisation
// (CGS2) for the Arnoldi step, and the Givens least-squares update, all on
// the device so that the host only polls a flag.
//
// Reductions: every block writes its partial sums; the last block to finish
// (atomic ticket) adds the partials in block order and resets the ticket, so
// results are bitwise reproducible for a given grid.
#include <cmath>

#include "internal.h"

namespace frjf {

constexpr int kChunk = 16;  // vectors per CGS dot-product pass

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sum of one accumulator; thread 0 receives the result.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kRedThreads / 64];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
#pragma unroll
    for (int w = 0; w < kRedThreads / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

int red_blocks(size_t n) {
  const size_t b = (n + (size_t)kRedThreads - 1) / (size_t)kRedThreads;
  return (int)std::max<size_t>(1, std::min<size_t>(b, kRedBlocks));
}

// out[i] = sum_b partials[b*stride + i], i < nv: one wavefront per output value, its
// lanes striding over the blocks, then a fixed-order wavefront tree (deterministic).
__global__ void __launch_bounds__(kRedThreads) k_finalize(const double* __restrict__ partials, int nblocks, int stride,
                                                          int nv, double* out, const int* skip) {
  if (skip != nullptr && *skip) return;
  const int i = blockIdx.x * (kRedThreads / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= nv) return;
  // all loads of a lane issued together (up to 16 per lane, kRedBlocks = 1024)
  double a[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int b = lane + 64 * q;
    a[q] = (b < nblocks) ? partials[(size_t)b * stride + i] : 0.0;
  }
  double s = 0.0;
  for (int b = lane + 64 * 16; b < nblocks; b += 64) s += partials[(size_t)b * stride + i];
#pragma unroll
  for (int q = 0; q < 16; ++q) s += a[q];
  s = wave_sum(s);
  if (lane == 0) out[i] = s;
}

hipError_t launch_finalize(const double* partials, int nblocks, int stride, int nv, double* out, const int* skip,
                           hipStream_t s) {
  const int waves = kRedThreads / 64;
  hipLaunchKernelGGL(k_finalize, dim3((nv + waves - 1) / waves), dim3(kRedThreads), 0, s, partials, nblocks, stride,
                     nv, out, skip);
  return hipGetLastError();
}

// ---------------------------------------------------------------- norm
__global__ void __launch_bounds__(kRedThreads) k_norm2_part(const double* __restrict__ x, size_t n, double* partials,
                                                            const int* skip) {
  if (skip != nullptr && *skip) return;
  double acc = 0.0;
  for (size_t i = blockIdx.x * (size_t)kRedThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kRedThreads)
    acc = fma(x[i], x[i], acc);
  acc = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

hipError_t launch_norm2(const double* x, size_t n, double* partials, unsigned*, double* out, const int* skip,
                        hipStream_t s) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(k_norm2_part, dim3(nb), dim3(kRedThreads), 0, s, x, n, partials, skip);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(partials, nb, 1, 1, out, skip, s);
}

// ---------------------------------------------------------------- linear combination
struct LinComb {
  const double* x[8];
  double c[8];
};

__global__ void __launch_bounds__(256) k_lincomb(double* __restrict__ y, int k, LinComb lc, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int t = 0; t < k; ++t) s = fma(lc.c[t], lc.x[t][i], s);
    y[i] = s;
  }
}

hipError_t launch_lincomb(double* y, int k, const double* const* x, const double* c, size_t n, hipStream_t s) {
  LinComb lc{};
  for (int t = 0; t < k && t < 8; ++t) {
    lc.x[t] = x[t];
    lc.c[t] = c[t];
  }
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_lincomb, dim3(blocks ? blocks : 1), dim3(256), 0, s, y, k, lc, n);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_scale_dev(double* __restrict__ y, const double* __restrict__ x,
                                                   const double* alpha, int inv, size_t n, const int* skip) {
  if (skip != nullptr && *skip) return;
  const double a = inv ? 1.0 / *alpha : *alpha;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

hipError_t launch_scale_dev(double* y, const double* x, const double* alpha, int inv, size_t n, const int* skip,
                            hipStream_t s) {
  const unsigned blocks = (unsigned)red_blocks(n);
  hipLaunchKernelGGL(k_scale_dev, dim3(blocks ? blocks : 1), dim3(256), 0, s, y, x, alpha, inv, n, skip);
  return hipGetLastError();
}

// ---------------------------------------------------------------- CGS2 Arnoldi step
// dots: partials[b*(kMaxM+2) + t] = block b's share of <w, V_t>, t < nv; grid.y splits the
// vectors into chunks of kChunk (each chunk re-reads its slice of w).
__global__ void __launch_bounds__(kRedThreads) k_cgs_dots(const double* __restrict__ V, int nv,
                                                          const double* __restrict__ w, double* partials,
                                                          const int* skip, size_t n) {
  if (skip != nullptr && *skip) return;
  const int t0 = blockIdx.y * kChunk;
  const int cnt = min(kChunk, nv - t0);
  double acc[kChunk];
#pragma unroll
  for (int t = 0; t < kChunk; ++t) acc[t] = 0.0;
  for (size_t i = blockIdx.x * (size_t)kRedThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kRedThreads) {
    const double wi = w[i];
#pragma unroll
    for (int t = 0; t < kChunk; ++t)
      if (t < cnt) acc[t] = fma(wi, V[(size_t)(t0 + t) * n + i], acc[t]);
  }
  __shared__ double red[kRedThreads / 64][kChunk];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < kChunk; ++t) {
    const double s = wave_sum(acc[t]);
    if (lane == 0) red[wv][t] = s;
  }
  __syncthreads();
  if (threadIdx.x < cnt) {
    double s = 0.0;
    for (int q = 0; q < kRedThreads / 64; ++q) s += red[q][threadIdx.x];
    partials[(size_t)blockIdx.x * (kMaxM + 2) + t0 + threadIdx.x] = s;
  }
}

static hipError_t cgs_pass(const double* V, int nv, double* w, const double* h, double* partials, double* out,
                           const int* skip, size_t n, hipStream_t s);

hipError_t launch_cgs_dots(const double* V, int nv, const double* w, double* partials, unsigned*, double* out,
                           const int* skip, size_t n, hipStream_t s) {
  return cgs_pass(V, nv, const_cast<double*>(w), nullptr, partials, out, skip, n, s);
}

// w -= sum_t h[t] V_t (t < nv)
__global__ void __launch_bounds__(256) k_cgs_update(const double* __restrict__ V, int nv, double* __restrict__ w,
                                                    const double* __restrict__ h, const int* skip, size_t n) {
  if (skip != nullptr && *skip) return;
  __shared__ double sh[kMaxM + 2];
  if (threadIdx.x < nv) sh[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double s = w[i];
    for (int t = 0; t < nv; ++t) s = fma(-sh[t], V[(size_t)t * n + i], s);
    w[i] = s;
  }
}

// Fused CGS pass: w -= sum_t h[t] V_t (if h) and partial sums of <w, V_t>, reading each
// V_t once; V_t(i) held in registers (NV >= nv, compile-time).
template <int NV>
__global__ void __launch_bounds__(kRedThreads) k_cgs_pass(const double* __restrict__ V, int nv, double* __restrict__ w,
                                                          const double* __restrict__ h, double* partials,
                                                          const int* skip, size_t n) {
  if (skip != nullptr && *skip) return;
  __shared__ double sh[NV];
  if (threadIdx.x < NV) sh[threadIdx.x] = (h != nullptr && threadIdx.x < nv) ? h[threadIdx.x] : 0.0;
  __syncthreads();
  double acc[NV];
#pragma unroll
  for (int t = 0; t < NV; ++t) acc[t] = 0.0;
  for (size_t i = blockIdx.x * (size_t)kRedThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kRedThreads) {
    double vr[NV];
#pragma unroll
    for (int t = 0; t < NV; ++t) vr[t] = (t < nv) ? V[(size_t)t * n + i] : 0.0;
    double s = w[i];
    if (h != nullptr) {
#pragma unroll
      for (int t = 0; t < NV; ++t) s = fma(-sh[t], vr[t], s);
      w[i] = s;
    }
#pragma unroll
    for (int t = 0; t < NV; ++t) acc[t] = fma(s, vr[t], acc[t]);
  }
  __shared__ double red[kRedThreads / 64][NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < NV; ++t) {
    const double r = wave_sum(acc[t]);
    if (lane == 0) red[wv][t] = r;
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    double r = 0.0;
    for (int q = 0; q < kRedThreads / 64; ++q) r += red[q][threadIdx.x];
    partials[(size_t)blockIdx.x * (kMaxM + 2) + threadIdx.x] = r;
  }
}

static hipError_t cgs_pass(const double* V, int nv, double* w, const double* h, double* partials, double* out,
                           const int* skip, size_t n, hipStream_t s) {
  const int nb = red_blocks(n);
  if (nv <= 8)
    hipLaunchKernelGGL(k_cgs_pass<8>, dim3(nb), dim3(kRedThreads), 0, s, V, nv, w, h, partials, skip, n);
  else if (nv <= 16)
    hipLaunchKernelGGL(k_cgs_pass<16>, dim3(nb), dim3(kRedThreads), 0, s, V, nv, w, h, partials, skip, n);
  else if (nv <= 24)
    hipLaunchKernelGGL(k_cgs_pass<24>, dim3(nb), dim3(kRedThreads), 0, s, V, nv, w, h, partials, skip, n);
  else if (nv <= 32)
    hipLaunchKernelGGL(k_cgs_pass<32>, dim3(nb), dim3(kRedThreads), 0, s, V, nv, w, h, partials, skip, n);
  else {
    // long restarts: plain update, then the chunked dot kernel
    if (h != nullptr) hipLaunchKernelGGL(k_cgs_update, dim3(nb), dim3(256), 0, s, V, nv, w, h, skip, n);
    hipLaunchKernelGGL(k_cgs_dots, dim3(nb, (nv + kChunk - 1) / kChunk), dim3(kRedThreads), 0, s, V, nv, w, partials,
                       skip, n);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(partials, nb, kMaxM + 2, nv, out, skip, s);
}

hipError_t launch_cgs_update_dots(const double* V, int nv, double* w, const double* h, double* partials,
                                  unsigned*, double* out, const int* skip, size_t n, hipStream_t s) {
  return cgs_pass(V, nv, w, h, partials, out, skip, n, s);
}

// Second update fused with the partial sums of ||w||^2.
__global__ void __launch_bounds__(kRedThreads) k_cgs_update_norm(const double* __restrict__ V, int nv,
                                                                 double* __restrict__ w, const double* __restrict__ h2,
                                                                 double* partials, const int* skip, size_t n) {
  if (*skip) return;
  __shared__ double sh[kMaxM + 2];
  if (threadIdx.x < nv) sh[threadIdx.x] = h2[threadIdx.x];
  __syncthreads();
  double acc = 0.0;
  for (size_t i = blockIdx.x * (size_t)kRedThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kRedThreads) {
    double s = w[i];
    for (int t = 0; t < nv; ++t) s = fma(-sh[t], V[(size_t)t * n + i], s);
    w[i] = s;
    acc = fma(s, s, acc);
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// One workgroup: ||w||^2 from the partials, then the Hessenberg column, the Givens
// rotations and the stop decision of Arnoldi step j = st->j; the status block is
// also written to mapped host memory for the host's poll.
__global__ void __launch_bounds__(kRedThreads) k_givens(GmState* st, const double* __restrict__ partials, int nblocks,
                                                        int M) {
  if (st->stop) return;
  __shared__ double col[kMaxM + 2], cs[kMaxM], sn[kMaxM];
  const int tid = threadIdx.x;
  const int j = st->j;
  const int ld = M + 1;
  if (tid <= j) col[tid] = st->h1[tid] + st->h2[tid];
  if (tid < j) {
    cs[tid] = st->cs[tid];
    sn[tid] = st->sn[tid];
  }
  double s = 0.0;
  for (int b = tid; b < nblocks; b += kRedThreads) s += partials[b];
  const double hn2 = block_sum(s);  // (contains barriers: the staged column is visible below)
  if (tid == 0) {
    const double hn = sqrt(hn2);
    double w02 = hn2;  // ||w||^2 before orthogonalisation (Pythagoras)
    for (int i = 0; i <= j; ++i) w02 += col[i] * col[i];
    st->w0 = sqrt(w02);
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      const double t = cs[i] * col[i] + sn[i] * col[i + 1];
      col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
      col[i] = t;
    }
    const double den = hypot(col[j], col[j + 1]);
    st->cs[j] = col[j] / den;
    st->sn[j] = col[j + 1] / den;
    col[j] = den;
    col[j + 1] = 0.0;
    st->g[j + 1] = -st->sn[j] * st->g[j];
    st->g[j] = st->cs[j] * st->g[j];
    const double rest = fabs(st->g[j + 1]);
    st->rest = rest;
    st->hn = hn;
    st->j = j + 1;
    if (!(rest == rest) || !(den == den) || isinf(rest) || den == 0.0) {
      st->stop = 1;
      st->why = 3;
    } else if (rest <= st->target) {
      st->stop = 1;
      st->why = 1;
    } else if (hn <= 1e-14 * st->w0) {
      st->stop = 1;
      st->why = 2;
    }
    GmStatus* hs = st->hslot;
    if (hs != nullptr) {
      hs->rest = st->rest;
      hs->beta = st->beta;
      hs->j = st->j;
      hs->stop = st->stop;
      hs->why = st->why;
    }
  }
  __syncthreads();
  if (tid <= j + 1) st->H[(size_t)j * ld + tid] = col[tid];
}

hipError_t launch_cgs_update_norm(const double* V, int nv, double* w, const double* h2, double* partials,
                                  unsigned*, GmState* st, int M, size_t n, hipStream_t s) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(k_cgs_update_norm, dim3(nb), dim3(kRedThreads), 0, s, V, nv, w, h2, partials, &st->stop, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(kRedThreads), 0, s, st, partials, nb, M);
  return hipGetLastError();
}

__global__ void k_gm_init(GmState* st, const double* beta2, double target, int M, GmStatus* hslot) {
  if (threadIdx.x != 0) return;
  st->hslot = hslot;
  const double beta = sqrt(*beta2);
  for (int i = 0; i <= M; ++i) st->g[i] = 0.0;
  st->g[0] = beta;
  st->beta = beta;
  st->target = target;
  st->j = 0;
  st->stop = 0;
  st->why = 0;
  st->rest = beta;
}

hipError_t launch_gm_init(GmState* st, const double* beta2, double target, int M, GmStatus* hslot, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_init, dim3(1), dim3(64), 0, s, st, beta2, target, M, hslot);
  return hipGetLastError();
}

// y = H(0:k,0:k)^{-1} g(0:k) by back substitution (upper triangular after the rotations)
__global__ void k_gm_solve_y(GmState* st, int k, int M) {
  if (threadIdx.x != 0) return;
  const int ld = M + 1;
  for (int i = k - 1; i >= 0; --i) {
    double s = st->g[i];
    for (int c = i + 1; c < k; ++c) s -= st->H[(size_t)c * ld + i] * st->y[c];
    st->y[i] = s / st->H[(size_t)i * ld + i];
  }
}

hipError_t launch_gm_solve_y(GmState* st, int k, int M, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_solve_y, dim3(1), dim3(64), 0, s, st, k, M);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_gm_update_x(double* __restrict__ x, const double* __restrict__ Z, int k,
                                                     const GmState* st, size_t n) {
  __shared__ double sy[kMaxM];
  if (threadIdx.x < k) sy[threadIdx.x] = st->y[threadIdx.x];
  __syncthreads();
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double s = x[i];
    for (int t = 0; t < k; ++t) s = fma(sy[t], Z[(size_t)t * n + i], s);
    x[i] = s;
  }
}

hipError_t launch_gm_update_x(double* x, const double* Z, int k, const GmState* st, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_update_x, dim3(red_blocks(n)), dim3(256), 0, s, x, Z, k, st, n);
  return hipGetLastError();
}

}  // namespace frjf
