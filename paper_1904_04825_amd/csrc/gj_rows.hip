// Batched in-place inversion of the FP64 element-Jacobi blocks (Section 4.5).
//
// A block is N x N, column-major (entry (i, j) at j N + i), one workgroup per
// block, and row i lives in the registers of thread i for the whole inversion.
// Gauss-Jordan elimination is carried out as N Jordan exchanges with partial
// pivoting: step k takes as pivot the row p_k with the largest |a_{p,0}| among
// the rows not pivoted yet (no rows are moved), scales that row by 1/pivot and
// eliminates column 0 from the others.  Every row is shifted left by one in the
// same step, the new column (1/pivot on the pivot row, -a_{i,0}/pivot elsewhere)
// entering at the right, so each register keeps a fixed place and the step loop
// needs no run-time register indexing.  After N steps the array M holds the
// inverse up to the pivot order: (P^{-1})_{k, p_j} = M_{p_k, j}.
// Only the pivot row goes through LDS; the per-step arithmetic is one FMA per
// held entry.
#include "internal.h"

namespace frjf {

// x moved across lanes by a DPP pattern (lanes without a source keep their own value)
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, 0xf, false);
  const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, 0xf, false);
  return __longlong_as_double(((long long)hi2 << 32) | (unsigned)lo2);
}

// Maximum of x over the wave, returned to every lane: row shifts accumulate each
// 16-lane row into its last lane, row broadcasts combine the rows into lane 63.
__device__ __forceinline__ double wave_max(double x) {
  x = fmax(x, dpp_move<0x111, 0xf>(x));  // row_shr:1
  x = fmax(x, dpp_move<0x112, 0xf>(x));  // row_shr:2
  x = fmax(x, dpp_move<0x114, 0xf>(x));  // row_shr:4
  x = fmax(x, dpp_move<0x118, 0xf>(x));  // row_shr:8
  x = fmax(x, dpp_move<0x142, 0xa>(x));  // row_bcast:15 into rows 1 and 3
  x = fmax(x, dpp_move<0x143, 0xc>(x));  // row_bcast:31 into rows 2 and 3
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int N, int NT>
__global__ void __launch_bounds__(NT) k_gj_rows(double* __restrict__ blocks) {
  constexpr int NW = NT / 64;
  __shared__ double rowp[N];   // the pivot row of the current step
  __shared__ double wbest[NW];
  __shared__ int wrow[NW];
  __shared__ int pivs[N];      // pivot row of every step
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double* A = blocks + (size_t)blockIdx.x * N * N;
  const bool own = tid < N;
  double a[N];
#pragma unroll
  for (int j = 0; j < N; ++j) a[j] = own ? A[(size_t)j * N + tid] : 0.0;
  int kstep = own ? -1 : N;  // step at which this row is the pivot; -1 while it is a candidate

  for (int k = 0; k < N; ++k) {
    // pivot: largest |a_{i,0}| over the candidate rows, ties to the lower row
    // (NaN entries never win the maximum; a wave whose candidates are all NaN still
    // offers its lowest candidate, a wave without candidates offers none)
    const bool cand = kstep < 0;
    const double mine = cand ? fabs(a[0]) : -1.0;
    double best = wave_max(mine);
    unsigned long long hit = __ballot(cand && mine == best);
    if (hit == 0) hit = __ballot(cand);
    if (hit == 0) best = -2.0;
    const int bi = w * 64 + (hit ? (int)__builtin_ctzll(hit) : 0);
    if (NW > 1 && lane == 0) {
      wbest[w] = best;
      wrow[w] = bi;
    }
    if (NW > 1) __syncthreads();
    int p = bi;
    if (NW > 1) {
      double b = wbest[0];
      p = wrow[0];
#pragma unroll
      for (int q = 1; q < NW; ++q)
        if (wbest[q] > b || (wbest[q] == b && wrow[q] < p)) {
          b = wbest[q];
          p = wrow[q];
        }
    }
    if (tid == p) {
#pragma unroll
      for (int j = 0; j < N; ++j) rowp[j] = a[j];
      kstep = k;
    }
    if (tid == 0) pivs[k] = p;
    __syncthreads();
    const double ipiv = 1.0 / rowp[0];
    // pivot row: a_j <- a_{j+1} / pivot, last <- 1/pivot; other rows:
    // a_j <- a_{j+1} - (a_0 / pivot) r_{j+1}, last <- -a_0 / pivot
    const bool is_p = tid == p;
    if (is_p) {
#pragma unroll
      for (int j = 0; j < N; ++j) a[j] = 0.0;
    }
    const double g = is_p ? -ipiv : a[0] * ipiv;
#pragma unroll
    for (int j = 0; j < N - 1; ++j) a[j] = fma(-g, rowp[j + 1], a[j + 1]);
    a[N - 1] = -g;
    // rowp is rewritten by the next step's pivot: with several waves the barrier of
    // the pivot search orders it, a single wave needs one here
    if (NW == 1) __syncthreads();
  }
  // (P^{-1})_{k_r, p_j} = M_{r, j}: thread r writes row k_r of the inverse
  if (own && kstep >= 0 && kstep < N) {
#pragma unroll
    for (int j = 0; j < N; ++j) A[(size_t)min(max(pivs[j], 0), N - 1) * N + kstep] = a[j];
  }
}

hipError_t launch_gj_rows_f64(int nb, double* blocks, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  switch (nb) {
    case 36:
      hipLaunchKernelGGL((k_gj_rows<36, 64>), dim3(nblk), dim3(64), 0, s, blocks);
      break;
    case 64:
      hipLaunchKernelGGL((k_gj_rows<64, 64>), dim3(nblk), dim3(64), 0, s, blocks);
      break;
    case 100:
      hipLaunchKernelGGL((k_gj_rows<100, 128>), dim3(nblk), dim3(128), 0, s, blocks);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace frjf
