// Batched in-place inversion of the large element-Jacobi blocks (Section 4.5) of the
// high-degree discretisations: N = 4 (P+1)^2 = 144 (P = 5) and 196 (P = 6), FP64 or
// FP32, column-major (entry (i, j) at j N + i), one workgroup per block.
//
// A block row does not fit one thread's registers, so the columns are cut into S
// segments of CS columns: thread (s, i) holds columns s CS .. s CS + CS - 1 of row i
// for the whole inversion (threads s RW .. s RW + RW - 1, RW = N rounded up to whole
// wavefronts, form segment s).  Gauss-Jordan elimination runs as N in-place Jordan
// exchanges with partial pivoting (no rows are moved): step k takes as pivot the row
// p with the largest |a_{p,k}| among the rows not pivoted yet; with f_i = a_{i,k} and
// r_j = a_{p,j}/a_{p,k} (r_k = 1/a_{p,k}) every entry becomes
//   row p:      a_{p,j} <- r_j,
//   row i != p: a_{i,j} <- a_{i,j} - f_i r_j   (a_{i,k} taken as 0),
// one FMA per held entry.  After N steps the array M holds the inverse up to the
// pivot order, (P^{-1})_{k, p_j} = M_{p_k, j}, undone on the way out.
// Per step: the segment that owns column k offers its candidates (a 64-bit key of
// |a| with the row in its low byte, one wavefront maximum each) and column k, then the
// pivot row goes through LDS; both LDS buffers alternate between even and odd steps,
// so two barriers per step suffice.  The step loop runs over segments at run time and
// over the segment's columns at compile time, so every register index is static.
#include "internal.h"

namespace frjf {

template <int N, int S, int U>
struct WideCfg {
  static constexpr int RW = (N + 63) / 64 * 64;  // threads per segment (whole wavefronts)
  static constexpr int CS = (N + S - 1) / S;     // columns per segment
  static constexpr int NT = S * RW;
  static constexpr int WPS = RW / 64;            // wavefronts per segment
  static_assert(N <= 256, "row index packed into one byte");
  static_assert(NT <= 1024, "one workgroup per block");
  static_assert(CS % U == 0 && S * CS == N, "whole step groups, no padding columns");
};

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long y = __shfl_xor(x, off, 64);
    x = y > x ? y : x;
  }
  return x;
}

// candidate key of row i with entry a: larger |a| first (ties and the low mantissa
// byte broken by the row), rows already pivoted 0
template <typename T>
__device__ __forceinline__ unsigned long long pivot_key(T a, int i, bool done) {
  if (done) return 0ull;
  if constexpr (sizeof(T) == 8) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(fabs((double)a));
    return (b & ~0xffull) | (unsigned long long)(255 - i);
  } else {
    const unsigned long long b = (unsigned long long)__float_as_uint(fabsf((float)a));
    return (b << 8) | (unsigned long long)(255 - i);
  }
}

// The step loop: U steps unrolled on compile-time register indices 0..U-1 of the owner
// segment, whose held columns rotate left by U after each such group (a[c] holds
// column s CS + (c + rot) mod CS of the row, rot = 0 outside the owner's turn; after
// its CS steps the owner is back in the original order).  All threads of a segment
// hold their columns in the same order, so the pivot row passes through LDS in that
// order and needs no index mapping.
template <typename T, int N, int S, int U>
__global__ void __launch_bounds__((WideCfg<N, S, U>::NT)) k_gj_wide(T* __restrict__ blocks) {
  using C = WideCfg<N, S, U>;
  constexpr int RW = C::RW, CS = C::CS, WPS = C::WPS;
  __shared__ T mcol[2][RW];                 // column k of every row
  __shared__ T prow[2][N];                  // the scaled pivot row
  __shared__ unsigned long long cand[2][WPS];
  __shared__ int perm[N];                   // pivot row of step k
  __shared__ int iperm[N];                  // step of pivot row i
  const int tid = threadIdx.x, s = tid / RW, i = tid - s * RW, lane = tid & 63, wseg = i >> 6;
  const bool live = i < N;
  T* A = blocks + (size_t)blockIdx.x * N * N;
  T a[CS];
#pragma unroll
  for (int c = 0; c < CS; ++c) a[c] = live ? A[(size_t)(s * CS + c) * N + i] : (T)0;
  bool done = !live;
#pragma unroll 1
  for (int sk = 0; sk < S; ++sk) {
    const bool owner = s == sk;
#pragma unroll 1
    for (int rot = 0; rot < CS; rot += U) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = sk * CS + rot + u;
        const int b = k & 1;
        // the owners of column k: candidates and the column
        if (owner) {
          const unsigned long long key = wave_max_u64(pivot_key(a[u], i, done));
          if (lane == 0) cand[b][wseg] = key;
          mcol[b][i] = a[u];
        }
        __syncthreads();
        unsigned long long best = cand[b][0];
#pragma unroll
        for (int w = 1; w < WPS; ++w) best = cand[b][w] > best ? cand[b][w] : best;
        const int p = 255 - (int)(best & 0xffull);
        const T rp = (T)1 / mcol[b][p];
        if (i == p) {
#pragma unroll
          for (int c = 0; c < CS; ++c) prow[b][s * CS + c] = (owner && c == u) ? rp : a[c] * rp;
          done = true;
        }
        if (tid == 0) perm[k] = p;
        __syncthreads();
        const T fi = mcol[b][i];
        const bool isp = i == p;
#pragma unroll
        for (int c = 0; c < CS; ++c) {
          const T rj = prow[b][s * CS + c];
          const T old = (owner && c == u) ? (T)0 : a[c];
          a[c] = isp ? rj : fma(-fi, rj, old);
          // a few pivot-row entries in flight at a time: hoisting more of them costs
          // registers the held row segment needs
          if (c % 8 == 7) asm volatile("" ::: "memory");
        }
      }
      if (owner) {
        T t[U];
#pragma unroll
        for (int c = 0; c < U; ++c) t[c] = a[c];
#pragma unroll
        for (int c = 0; c + U < CS; ++c) a[c] = a[c + U];
#pragma unroll
        for (int c = 0; c < U; ++c) a[CS - U + c] = t[c];
      }
    }
  }
  __syncthreads();
  for (int t = tid; t < N; t += C::NT) iperm[perm[t]] = t;
  __syncthreads();
  if (live) {
    const int row = iperm[i];
#pragma unroll
    for (int c = 0; c < CS; ++c) A[(size_t)perm[s * CS + c] * N + row] = a[c];
  }
}

// In-place inversion of nblk blocks of order nb (144 or 196), FP64 or FP32.
// Four segments (1024 or 768 threads): fewer, longer segments measured more register
// spills at compile time (the compiler keeps about twice the held entries live).
template <typename T, int N, int S, int U>
static void launch_wide_cfg(T* blocks, int nblk, hipStream_t s) {
  hipLaunchKernelGGL((k_gj_wide<T, N, S, U>), dim3(nblk), dim3(WideCfg<N, S, U>::NT), 0, s, blocks);
}

template <typename T>
static hipError_t launch_wide(int nb, T* blocks, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  switch (nb) {
    case 144:
      launch_wide_cfg<T, 144, 4, 6>(blocks, nblk, s);
      break;
    case 196:
      launch_wide_cfg<T, 196, 4, 7>(blocks, nblk, s);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gj_wide_f64(int nb, double* blocks, int nblk, hipStream_t s) {
  return launch_wide<double>(nb, blocks, nblk, s);
}
hipError_t launch_gj_wide_f32(int nb, float* blocks, int nblk, hipStream_t s) {
  return launch_wide<float>(nb, blocks, nblk, s);
}

}  // namespace frjf
