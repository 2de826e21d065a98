// Vector kernels of the GMRES layer (Section 4.5): deterministic norms,
// linear combinations, classical Gram-Schmidt with one re-orthogonalisation
// (CGS2) for the Arnoldi step, and the Givens least-squares update, all on
// the device so that the host only polls a flag.
//
// Reductions: every workgroup writes its partial sums, and a second kernel adds
// the partials in block order, so results are bitwise reproducible for a given
// grid.
#include <cmath>

#include "arnoldi.h"
#include "internal.h"
#include "wavesum.h"

namespace frjf {

constexpr int kChunk = 16;  // vectors per CGS dot-product pass

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

hipError_t launch_norm2_parts(const double* x, size_t n, double* partials, int* nb, const int* skip, hipStream_t s) {
  *nb = red_blocks(n);
  hipLaunchKernelGGL(k_norm2_part, dim3(*nb), dim3(kRedThreads), 0, s, x, n, partials, skip);
  return hipGetLastError();
}

hipError_t launch_norm2(const double* x, size_t n, double* partials, double* out, const int* skip,
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

// ---------------------------------------------------------------- CGS2 Arnoldi step
#ifndef FRJF_CGS_EPT
#define FRJF_CGS_EPT 4
#endif
// Workgroups of the CGS passes: at least FRJF_CGS_EPT entries per thread, so the
// partial sums of a workgroup cover enough of the vectors to pay for its reduction,
// and at most kRedBlocks (four waves per SIMD keep enough loads in flight on long
// vectors); every workgroup of the next pass adds all of them, with one load per
// thread and value up to kRedThreads workgroups.
int cgs_blocks(size_t n) {
  const size_t per = (size_t)kRedThreads * FRJF_CGS_EPT;
  return (int)std::max<size_t>(1, std::min<size_t>((n + per - 1) / per, kRedBlocks));
}

// dots: partials[b*kPartStride + t] = block b's share of <w, V_t>, t < nv; grid.y splits the
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
  const int wv = threadIdx.x >> 6;
  int off;
  if (wave_multi_sum<kChunk>(acc, off)) {
#pragma unroll
    for (int t = 0; t < multi_sum_count(kChunk); ++t) red[wv][off + t] = acc[t];
  }
  __syncthreads();
  if (threadIdx.x < cnt) {
    double s = 0.0;
    for (int q = 0; q < kRedThreads / 64; ++q) s += red[q][threadIdx.x];
    partials[(size_t)blockIdx.x * kPartStride + t0 + threadIdx.x] = s;
  }
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

// Fused CGS pass over V_0 .. V_{nv-1}, each read once, one partial sum per value and
// workgroup, stored at partials[t kRedBlocks + b] (value t, workgroup b):
//   h = the sums over b < hnb of the previous pass's partials hpart, when hpart is
//       given; every workgroup adds them in the same order, workgroup 0 stores h to
//       hout;
//   w -= sum_t h[t] V_t (when hpart is given);
//   partial sums of <w, V_t> (DOTS) or of ||w||^2 (!DOTS).
// NV >= nv is a multiple of 4 and every slot loads unconditionally, so the loads of
// an entry are issued together: the slots t >= nv re-read V_{nv-1} with weight 0,
// and their sums are dropped.  The first entry's loads are in flight while h is
// summed.  Requires hnb <= kRedBlocks.
template <int NV, bool DOTS>
__global__ void __launch_bounds__(kRedThreads) k_cgs_pass(const double* __restrict__ V, int nv, double* __restrict__ w,
                                                          const double* __restrict__ hpart, int hnb, double* hout,
                                                          double* __restrict__ partials, const int* skip, size_t n) {
  if (skip != nullptr && *skip) return;
  constexpr int NA = DOTS ? NV : 1;
  __shared__ double sh[NV];
  __shared__ double red[kRedThreads / 64][NV];
  const int tid = threadIdx.x, wv = tid >> 6;
  const size_t stride = (size_t)gridDim.x * kRedThreads;
  size_t i = blockIdx.x * (size_t)kRedThreads + tid;
  double vr[NV], wi = 0.0;
  auto load = [&](size_t k) {
#pragma unroll
    for (int t = 0; t < NV; ++t) vr[t] = V[(size_t)min(t, nv - 1) * n + k];
    wi = w[k];
  };
  if (i < n) load(i);
  if (hpart != nullptr) {
    double hr[NV];
#pragma unroll
    for (int t = 0; t < NV; ++t) hr[t] = (tid < hnb) ? hpart[(size_t)min(t, nv - 1) * kRedBlocks + tid] : 0.0;
    for (int b = tid + kRedThreads; b < hnb; b += kRedThreads) {
#pragma unroll
      for (int t = 0; t < NV; ++t) hr[t] += hpart[(size_t)min(t, nv - 1) * kRedBlocks + b];
    }
    int off;
    if (wave_multi_sum<NV>(hr, off)) {
#pragma unroll
      for (int t = 0; t < multi_sum_count(NV); ++t) red[wv][off + t] = hr[t];
    }
    __syncthreads();
    if (tid < NV) {
      double r = 0.0;
#pragma unroll
      for (int q = 0; q < kRedThreads / 64; ++q) r += red[q][tid];
      sh[tid] = tid < nv ? r : 0.0;
      if (blockIdx.x == 0 && tid < nv) hout[tid] = r;
    }
    __syncthreads();
  }
  double acc[NA];
#pragma unroll
  for (int t = 0; t < NA; ++t) acc[t] = 0.0;
  for (; i < n; i += stride) {
    double s = wi;
    if (hpart != nullptr) {
#pragma unroll
      for (int t = 0; t < NV; ++t) s = fma(-sh[t], vr[t], s);
      w[i] = s;
    }
    if constexpr (DOTS) {
#pragma unroll
      for (int t = 0; t < NV; ++t) acc[t] = fma(s, vr[t], acc[t]);
    } else {
      acc[0] = fma(s, s, acc[0]);
    }
    if (i + stride < n) load(i + stride);
  }
  int off;
  if (wave_multi_sum<NA>(acc, off)) {
#pragma unroll
    for (int t = 0; t < multi_sum_count(NA); ++t) red[wv][off + t] = acc[t];
  }
  __syncthreads();
  if (tid < (DOTS ? nv : 1)) {
    double r = 0.0;
#pragma unroll
    for (int q = 0; q < kRedThreads / 64; ++q) r += red[q][tid];
    partials[(size_t)tid * kRedBlocks + blockIdx.x] = r;
  }
}

// k_cgs_pass with NV = nv rounded up to a multiple of 4 (nv <= 32)
template <bool DOTS>
static void launch_cgs_pass(int nb, const double* V, int nv, double* w, const double* hpart, int hnb, double* hout,
                            double* partials, const int* skip, size_t n, hipStream_t s) {
  const dim3 g(nb), b(kRedThreads);
#define FRJF_CGS_CASE(K, NVV)                                                                                         \
  case K:                                                                                                             \
    hipLaunchKernelGGL((k_cgs_pass<NVV, DOTS>), g, b, 0, s, V, nv, w, hpart, hnb, hout, partials, skip, n);           \
    break;
  switch ((nv + 3) / 4) {
    FRJF_CGS_CASE(1, 4)
    FRJF_CGS_CASE(2, 8)
    FRJF_CGS_CASE(3, 12)
    FRJF_CGS_CASE(4, 16)
    FRJF_CGS_CASE(5, 20)
    FRJF_CGS_CASE(6, 24)
    FRJF_CGS_CASE(7, 28)
    FRJF_CGS_CASE(8, 32)
    default:
      break;
  }
#undef FRJF_CGS_CASE
}

// Second update fused with the partial sums of ||w||^2, for restarts longer than the
// register-held passes (nv > 32).
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

// One workgroup: the Givens update of Arnoldi step st->j on its own (the last step
// of a cycle; the others run it inside the next step's preconditioner kernel).
__global__ void __launch_bounds__(kRedThreads) k_givens(GmState* st, const double* __restrict__ partials, int nblocks,
                                                        int M) {
  if (st->stop) return;
  __shared__ GivensLds L;
  const double hn2 = block_sum_partials(partials, nblocks, L.red);
  givens_step(st, hn2, M, L);
}

hipError_t launch_givens(GmState* st, const double* norm_part, int nb, int M, hipStream_t s) {
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(kRedThreads), 0, s, st, norm_part, nb, M);
  return hipGetLastError();
}

hipError_t launch_arnoldi_cgs2(const double* V, int nv, double* w, double* partials, GmState* st, int M, size_t n,
                               hipStream_t s) {
  const int nb = cgs_blocks(n);
  const int* skip = &st->stop;
  double* P1 = partials;
  double* P2 = partials + kPartSecond;
  if (nv <= 32) {
    launch_cgs_pass<true>(nb, V, nv, w, nullptr, 0, nullptr, P1, skip, n, s);  // h1 = V^T w
    launch_cgs_pass<true>(nb, V, nv, w, P1, nb, st->h1, P2, skip, n, s);       // w -= V h1; h2 = V^T w
    launch_cgs_pass<false>(nb, V, nv, w, P2, nb, st->h2, P1, skip, n, s);      // w -= V h2; ||w||^2
  } else {
    // long restarts: chunked dot kernels with separate sums, the update kernels
    const dim3 gd(nb, (nv + kChunk - 1) / kChunk);
    hipError_t e;
    hipLaunchKernelGGL(k_cgs_dots, gd, dim3(kRedThreads), 0, s, V, nv, w, P1, skip, n);
    if ((e = launch_finalize(P1, nb, kPartStride, nv, st->h1, skip, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cgs_update, dim3(nb), dim3(kRedThreads), 0, s, V, nv, w, st->h1, skip, n);
    hipLaunchKernelGGL(k_cgs_dots, gd, dim3(kRedThreads), 0, s, V, nv, w, P1, skip, n);
    if ((e = launch_finalize(P1, nb, kPartStride, nv, st->h2, skip, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cgs_update_norm, dim3(nb), dim3(kRedThreads), 0, s, V, nv, w, st->h2, P1, skip, n);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- DCGS2 Arnoldi step
// Classical Gram-Schmidt with the re-orthogonalisation of each basis vector delayed
// to the next step, so both projections share the reads of V: at step j, V_0 ..
// V_{j-1} are final and V_j = ~v_j is the new vector, orthogonalised once and of unit
// norm; w = A z_j.
//   pass 1, one read of V and w:  b_t = <V_t, w> (t <= j), a_t = <V_t, ~v_j> (t < j),
//     <w, w>;
//   pass 2, every workgroup adds pass 1's partials, alpha = sqrt(1 - |a|^2) (Pythagoras:
//     ~v_j - V a is orthogonal to V_0 .. V_{j-1}), c_j = (b_j - a.b) / alpha, and for
//     every entry: v_j = (~v_j - sum_{t<j} a_t V_t) / alpha (stored over ~v_j),
//     w' = w - sum_{t<j} b_t V_t - c_j v_j, partial sums of ||w'||^2.  Workgroup 0
//     makes column j-1 final (h_{t,j-1} += h_{j,j-1} a_t, h_{j,j-1} *= alpha: the
//     correction of ~v_j expressed in the final basis), rotates it, and stores column
//     j's first pass (b_t, c_j) and ||w||.
// The next step's preconditioner kernel forms ~v_{j+1} = w' / ||w'||.

template <int NV>
__global__ void __launch_bounds__(kRedThreads) k_dcgs_dots(const double* __restrict__ V, int nv,
                                                           const double* __restrict__ w, double* __restrict__ partials,
                                                           const int* skip, size_t n) {
  if (*skip) return;
  constexpr int NA = 2 * NV;  // b_t at t, a_t at NV + t (t < NV - 1), <w, w> at 2 NV - 1
  __shared__ double red[kRedThreads / 64][NA];
  const int tid = threadIdx.x, wv = tid >> 6;
  const double* vj = V + (size_t)(nv - 1) * n;
  double acc[NA];
#pragma unroll
  for (int t = 0; t < NA; ++t) acc[t] = 0.0;
  // the next entry's loads are issued before this entry's FMAs (one round trip per
  // entry hidden behind the previous one)
  const size_t stride = (size_t)gridDim.x * kRedThreads;
  size_t i = (size_t)xcd_remap(blockIdx.x, gridDim.x) * kRedThreads + tid;
  double vr[NV], wi = 0.0, vji = 0.0;
  auto load = [&](size_t k) {
#pragma unroll
    for (int t = 0; t < NV; ++t) vr[t] = V[(size_t)min(t, nv - 1) * n + k];
    wi = w[k];
    vji = vj[k];
  };
  if (i < n) load(i);
  for (; i < n; i += stride) {
    double cr[NV];
#pragma unroll
    for (int t = 0; t < NV; ++t) cr[t] = vr[t];
    const double cw = wi, cj = vji;
    if (i + stride < n) load(i + stride);
#pragma unroll
    for (int t = 0; t < NV; ++t) acc[t] = fma(cr[t], cw, acc[t]);
#pragma unroll
    for (int t = 0; t + 1 < NV; ++t) acc[NV + t] = fma(cr[t], cj, acc[NV + t]);
    acc[NA - 1] = fma(cw, cw, acc[NA - 1]);
  }
  int off;
  if (wave_multi_sum<NA>(acc, off)) {
#pragma unroll
    for (int t = 0; t < multi_sum_count(NA); ++t) red[wv][off + t] = acc[t];
  }
  __syncthreads();
  if (tid < NA) {
    double r = 0.0;
#pragma unroll
    for (int q = 0; q < kRedThreads / 64; ++q) r += red[q][tid];
    partials[(size_t)tid * kRedBlocks + blockIdx.x] = r;
  }
}

template <int NV>
__global__ void __launch_bounds__(kRedThreads) k_dcgs_update(double* __restrict__ V, int nv, double* __restrict__ w,
                                                             const double* __restrict__ part1, int nb,
                                                             double* __restrict__ normpart, GmState* st, int M,
                                                             size_t n) {
  if (st->stop) return;
  constexpr int NA = 2 * NV;
  __shared__ double red[kRedThreads / 64][NA];
  __shared__ double val[NA];
  __shared__ double sa[NV], sb[NV], sc[3];
  __shared__ GivensLds L;
  const int tid = threadIdx.x, wv = tid >> 6;
  const int j = nv - 1;
  double* vj = V + (size_t)j * n;
  const size_t stride = (size_t)gridDim.x * kRedThreads;
  size_t i = (size_t)xcd_remap(blockIdx.x, gridDim.x) * kRedThreads + tid;
  double vr[NV], wi = 0.0, vji = 0.0;
  auto load = [&](size_t k) {
#pragma unroll
    for (int t = 0; t < NV; ++t) vr[t] = V[(size_t)min(t, nv - 1) * n + k];
    wi = w[k];
    vji = vj[k];
  };
  if (i < n) load(i);
  // pass 1's sums, the same in every workgroup
  {
    double hr[NA];
#pragma unroll
    for (int t = 0; t < NA; ++t) hr[t] = (tid < nb) ? part1[(size_t)t * kRedBlocks + tid] : 0.0;
    for (int b = tid + kRedThreads; b < nb; b += kRedThreads) {
#pragma unroll
      for (int t = 0; t < NA; ++t) hr[t] += part1[(size_t)t * kRedBlocks + b];
    }
    int off;
    if (wave_multi_sum<NA>(hr, off)) {
#pragma unroll
      for (int t = 0; t < multi_sum_count(NA); ++t) red[wv][off + t] = hr[t];
    }
    __syncthreads();
    if (tid < NA) {
      double r = 0.0;
#pragma unroll
      for (int q = 0; q < kRedThreads / 64; ++q) r += red[q][tid];
      val[tid] = r;
    }
    __syncthreads();
  }
  if (tid == 0) {
    double aa = 0.0, ab = 0.0;
    for (int t = 0; t < j; ++t) {
      aa = fma(val[NV + t], val[NV + t], aa);
      ab = fma(val[NV + t], val[t], ab);
    }
    const double alpha2 = 1.0 - aa;
    const double alpha = alpha2 > 0.0 ? sqrt(alpha2) : 0.0;  // 0: ~v_j in the span of V (breakdown)
    sc[0] = alpha;
    sc[1] = alpha > 0.0 ? 1.0 / alpha : 0.0;
    sc[2] = alpha > 0.0 ? (val[j] - ab) / alpha : 0.0;
  }
  if (tid < NV) {
    sa[tid] = tid < j ? val[NV + tid] : 0.0;
    sb[tid] = tid < j ? val[tid] : 0.0;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    if (j >= 1) {
      const double hn = st->hn;  // first-pass h_{j,j-1} = ||w'|| of step j-1
      if (tid < j) L.col[tid] = st->h1[tid] + hn * sa[tid];
      if (tid == 0) L.col[j] = hn * sc[0];
      load_rotations(st, j - 1, L);
      __syncthreads();
      if (tid == 0) givens_rotate(st, j - 1, L.col, L.cs, L.sn, st->w0);
      __syncthreads();
      store_column(st, j - 1, M, L);
      __syncthreads();
    }
    if (tid < j) st->h1[tid] = val[tid];
    if (tid == 0) {
      st->h1[j] = sc[2];
      st->w0 = sqrt(val[NA - 1]);
      st->evals = j + 1;  // this step's JF product ran
    }
  }
  const double ia = sc[1], cj = sc[2];
  double acc = 0.0;
  for (; i < n; i += stride) {
    double s = vji;
#pragma unroll
    for (int t = 0; t < NV; ++t) s = fma(-sa[t], vr[t], s);
    const double vn = s * ia;
    if (j >= 1) vj[i] = vn;
    double u = wi;
#pragma unroll
    for (int t = 0; t < NV; ++t) u = fma(-sb[t], vr[t], u);
    u = fma(-cj, vn, u);
    w[i] = u;
    acc = fma(u, u, acc);
    if (i + stride < n) load(i + stride);
  }
  acc = wave_sum(acc);
  if ((tid & 63) == 0) red[wv][0] = acc;
  __syncthreads();
  if (tid == 0) {
    double r = 0.0;
#pragma unroll
    for (int q = 0; q < kRedThreads / 64; ++q) r += red[q][0];
    normpart[blockIdx.x] = r;
  }
}

// The cycle's last column, first pass as it stands, with ||w'|| from the last pass 2.
__global__ void __launch_bounds__(kRedThreads) k_dcgs_last(GmState* st, const double* __restrict__ normpart, int nb,
                                                           int M) {
  if (st->stop) return;
  __shared__ GivensLds L;
  const double hn2 = block_sum_partials(normpart, nb, L.red);
  givens_first_pass(st, sqrt(hn2), M, L);
}

bool dcgs2_supported(int m) { return m <= 32; }

// which: 1 the first pass, 2 the second (its partial rows from nb1 workgroups), 3 both
static hipError_t dcgs2_passes(int which, double* V, int nv, double* w, double* partials, int nb1, GmState* st,
                               int M, size_t n, hipStream_t s) {
  const int nb = cgs_blocks(n);
  if (which == 3) nb1 = nb;
  if (nb1 < 1 || nb1 > kRedBlocks) return hipErrorInvalidValue;
  double* np = partials + kDcgsNormOff;
  const dim3 g(nb), b(kRedThreads);
#define FRJF_DCGS_CASE(K, NVV)                                                                                      \
  case K:                                                                                                           \
    if (which & 1) hipLaunchKernelGGL((k_dcgs_dots<NVV>), g, b, 0, s, V, nv, w, partials, &st->stop, n);           \
    if (which & 2) hipLaunchKernelGGL((k_dcgs_update<NVV>), g, b, 0, s, V, nv, w, partials, nb1, np, st, M, n);    \
    break;
  switch ((nv + 3) / 4) {
    FRJF_DCGS_CASE(1, 4)
    FRJF_DCGS_CASE(2, 8)
    FRJF_DCGS_CASE(3, 12)
    FRJF_DCGS_CASE(4, 16)
    FRJF_DCGS_CASE(5, 20)
    FRJF_DCGS_CASE(6, 24)
    FRJF_DCGS_CASE(7, 28)
    FRJF_DCGS_CASE(8, 32)
    default:
      return hipErrorInvalidValue;
  }
#undef FRJF_DCGS_CASE
  return hipGetLastError();
}

hipError_t launch_arnoldi_dcgs2(double* V, int nv, double* w, double* partials, GmState* st, int M, size_t n,
                                hipStream_t s) {
  return dcgs2_passes(3, V, nv, w, partials, 0, st, M, n, s);
}

hipError_t launch_dcgs2_update(double* V, int nv, double* w, double* partials, int nb1, GmState* st, int M,
                               size_t n, hipStream_t s) {
  return dcgs2_passes(2, V, nv, w, partials, nb1, st, M, n, s);
}

const double* dcgs2_norm_partials(const double* partials) { return partials + kDcgsNormOff; }

hipError_t launch_dcgs2_last(GmState* st, const double* partials, int nb, int M, hipStream_t s) {
  hipLaunchKernelGGL(k_dcgs_last, dim3(1), dim3(kRedThreads), 0, s, st, partials + kDcgsNormOff, nb, M);
  return hipGetLastError();
}

// Start of a restart cycle: every workgroup forms beta = ||r|| from ||r||^2 and stores
// the first basis vector v_0 = r / beta; workgroup 0 also resets the cycle state.
// Start of a restart cycle: every workgroup forms beta = ||r|| from ||r||^2 and stores
// the first basis vector v_0 = r / beta; workgroup 0 also resets the cycle state.  The
// solve's first cycle also sets the reference norm (ref, or beta when ref <= 0), the
// target rtol * r_ref and the totals, and ends the solve before any step when beta is
// not finite or already at the target.  A later cycle does nothing once the solve ended.
__global__ void __launch_bounds__(256) k_gm_start(GmState* st, const double* beta2, double rtol, double ref, int M,
                                                  GmStatus* hslot, double* __restrict__ v0,
                                                  const double* __restrict__ r, size_t n, int first) {
  if (!first && st->fz.fin) return;
  const double beta = sqrt(*beta2);
  const double r_ref = ref > 0.0 ? ref : beta;
  const double target = first ? rtol * r_ref : st->target;
  const bool end0 = first && (!isfinite(beta) || beta <= target);
  if (!end0) {
    const double a = 1.0 / beta;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
      v0[i] = a * r[i];
  }
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  if (first) {
    st->fz.fin = 0;
    st->fz.result = FR_NOTCONV;
    st->fz.iters = 0;
    st->fz.evals = 0;
    st->fz.steps = 0;
    st->fz.restarts = 0;
    st->fz.r_final = beta;
    st->fz.r_ref = r_ref;
    st->target = target;
  }
  st->hslot = hslot;
  for (int i = 0; i <= M; ++i) st->g[i] = 0.0;
  st->g[0] = beta;
  st->beta = beta;
  st->j = 0;
  st->stop = 0;
  st->why = 0;
  st->evals = 0;
  st->done = 0;
  st->rest = beta;
  if (end0) {
    st->fz.fin = 1;
    st->fz.result = isfinite(beta) ? FR_OK : FR_ENAN;
    st->stop = 1;
    st->done = 1;
    if (hslot != nullptr) hslot->stop = 1;
  }
}

hipError_t launch_gm_start(GmState* st, const double* beta2, double rtol, double ref, int M, GmStatus* hslot,
                           double* v0, const double* r, size_t n, int first, hipStream_t s) {
  const unsigned blocks = (unsigned)red_blocks(n);
  hipLaunchKernelGGL(k_gm_start, dim3(blocks ? blocks : 1), dim3(256), 0, s, st, beta2, rtol, ref, M, hslot, v0, r,
                     n, first);
  return hipGetLastError();
}

// One thread: the cycle's steps and JF products into the totals (DCGS2 finds
// convergence one step late: the product of that step also ran), then NaN or
// convergence of the least-squares residual end the solve; otherwise the restart's
// true residual (one more product) decides: NaN, converged, breakdown, or the
// iteration limit end it, else the solve restarts.  An end stops every later kernel
// and is mirrored to the mapped host status.
__global__ void __launch_bounds__(64) k_gm_cycle_end(GmState* st, double* beta2, const double* opart, int nbo,
                                                     int max_iters, int dcgs) {
  if (st->fz.fin) return;
  // ||r||^2 from the true residual's partial sums (one wavefront, fixed order) when given
  double b2 = 0.0;
  if (opart != nullptr) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nbo; b += 64) v += opart[b];
    b2 = wave_sum(v);
  }
  if (threadIdx.x != 0) return;
  if (opart != nullptr)
    *beta2 = b2;  // the next cycle's start reads it
  else
    b2 = *beta2;
  const int k = st->j, why = st->why;
  st->fz.iters += k;
  st->fz.evals += dcgs ? max(k, st->evals) : k;
  st->fz.steps += dcgs ? max(k, st->evals) : k;
  double rf = st->rest;
  int res = -1;
  if (why == 3) {
    res = FR_ENAN;
  } else if (why == 1) {
    res = FR_OK;
  } else {
    st->fz.evals += 1;
    const double beta = sqrt(b2);
    rf = beta;
    if (!isfinite(beta))
      res = FR_ENAN;
    else if (beta <= st->target)
      res = FR_OK;
    else if (why == 2)
      res = FR_BREAKDOWN;
    else if (st->fz.iters >= max_iters)
      res = FR_NOTCONV;
    else
      st->fz.restarts += 1;
  }
  st->fz.r_final = rf;
  if (res >= 0) {
    st->fz.fin = 1;
    st->fz.result = res;
    st->stop = 1;
    st->done = 1;
    if (st->hslot != nullptr) st->hslot->stop = 1;
  }
}

hipError_t launch_gm_cycle_end(GmState* st, const double* beta2, int max_iters, int dcgs, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_cycle_end, dim3(1), dim3(64), 0, s, st, const_cast<double*>(beta2), nullptr, 0, max_iters,
                     dcgs);
  return hipGetLastError();
}

hipError_t launch_gm_cycle_end_parts(GmState* st, double* beta2, const double* opart, int nbo, int max_iters,
                                     int dcgs, hipStream_t s) {
  if (opart == nullptr || nbo < 1 || nbo > kRedBlocks) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gm_cycle_end, dim3(1), dim3(64), 0, s, st, beta2, opart, nbo, max_iters, dcgs);
  return hipGetLastError();
}

// End of a cycle: x += sum_t y_t Z_t with y = H(0:k,0:k)^{-1} g(0:k), k = st->j (H is
// upper triangular after the rotations), and per-workgroup partial sums of ||x||^2 for
// the epsilon of the restart's true residual.  Every workgroup solves the small system
// itself: all threads stage the triangle in LDS ([column][row]), then one wavefront
// back-substitutes (lane i holds the right-hand side of row i; column c's
// y_c = r_c / R_cc is broadcast and removed from the rows above it) while the first
// entries of Z are on their way.  NV > 0: the k <= NV columns of an entry loaded
// together (slots t >= k re-read column k-1 with weight 0); NV = 0: a plain loop.
// After NaN (why = 3), with k = 0 or once the solve has ended, x is left as it is.
template <int NV>
__global__ void __launch_bounds__(256) k_gm_update_x(double* __restrict__ x, const double* __restrict__ Z,
                                                     const GmState* st, int M, size_t n, double* __restrict__ xpart) {
  __shared__ double R[kMaxM][kMaxM + 1];
  __shared__ double sy[kMaxM];
  __shared__ double red[4];
  const int k = st->j;
  const bool upd = !(st->fz.fin || st->why == 3 || k <= 0);
  const int tid = threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = blockIdx.x * (size_t)blockDim.x + tid;
  double zr[NV > 0 ? NV : 1];
  if constexpr (NV > 0) {
    if (upd && i < n) {
#pragma unroll
      for (int t = 0; t < NV; ++t) zr[t] = Z[(size_t)min(t, k - 1) * n + i];
    }
  }
  if (upd) {
    const int ld = M + 1;
    for (int idx = tid; idx < k * k; idx += blockDim.x) {
      const int c = idx / k, r = idx - c * k;
      if (r <= c) R[c][r] = st->H[(size_t)c * ld + r];
    }
    if (tid < kMaxM) sy[tid] = 0.0;
    __syncthreads();
    if (tid < 64) {
      double r = tid < k ? st->g[tid] : 0.0;
      for (int c = k - 1; c >= 0; --c) {
        const int lo = __builtin_amdgcn_readlane(__double2loint(r), c), hi = __builtin_amdgcn_readlane(__double2hiint(r), c);
        const double yc = __hiloint2double(hi, lo) / R[c][c];
        if (tid == c) sy[c] = yc;
        if (tid < c) r = fma(-R[c][tid], yc, r);
      }
    }
    __syncthreads();
  }
  double acc = 0.0;
  for (; i < n; i += stride) {
    double s = x[i];
    if (upd) {
      if constexpr (NV > 0) {
#pragma unroll
        for (int t = 0; t < NV; ++t) s = fma(sy[t], zr[t], s);
        if (i + stride < n) {
#pragma unroll
          for (int t = 0; t < NV; ++t) zr[t] = Z[(size_t)min(t, k - 1) * n + i + stride];
        }
      } else {
        for (int t = 0; t < k; ++t) s = fma(sy[t], Z[(size_t)t * n + i], s);
      }
      x[i] = s;
    }
    acc = fma(s, s, acc);
  }
  acc = wave_sum(acc);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) xpart[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t launch_gm_update_x(double* x, const double* Z, int M, const GmState* st, size_t n, double* xpart,
                              int* nb_out, hipStream_t s) {
  if (M < 1 || M > kMaxM) return hipErrorInvalidValue;
  const int nb = red_blocks(n);
  *nb_out = nb;
  const dim3 g(nb), b(256);
  if (M <= 8)
    hipLaunchKernelGGL((k_gm_update_x<8>), g, b, 0, s, x, Z, st, M, n, xpart);
  else if (M <= 16)
    hipLaunchKernelGGL((k_gm_update_x<16>), g, b, 0, s, x, Z, st, M, n, xpart);
  else if (M <= 24)
    hipLaunchKernelGGL((k_gm_update_x<24>), g, b, 0, s, x, Z, st, M, n, xpart);
  else if (M <= 32)
    hipLaunchKernelGGL((k_gm_update_x<32>), g, b, 0, s, x, Z, st, M, n, xpart);
  else
    hipLaunchKernelGGL((k_gm_update_x<0>), g, b, 0, s, x, Z, st, M, n, xpart);
  return hipGetLastError();
}

}  // namespace frjf
