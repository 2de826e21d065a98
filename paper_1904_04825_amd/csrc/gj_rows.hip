// Batched in-place inversion of the FP64 element-Jacobi blocks (Section 4.5).
//
// A block is N x N, column-major (entry (i, j) at j N + i), one workgroup per
// block, and row i lives in the registers of thread i for the whole inversion.
// Gauss-Jordan elimination is carried out as N in-place Jordan exchanges with
// partial pivoting: step k takes as pivot the row p_k with the largest |a_{p,c}|
// in the step's column c among the rows not pivoted yet (no rows are moved) and
// eliminates column c from the others; column c then holds the new column of the
// inverse (-a_{i,c}/pivot).  The pivot row is not scaled in the loop: it keeps its
// entries, a 1 in column c, and the factor 1/pivot, applied once at the end.  A
// row's later updates are linear in the row, so a pending factor commutes with
// them.  U steps are unrolled with compile-time columns 0..U-1; between such groups
// every row is rotated left by U, so the step loop needs no run-time register
// indexing and the rotation costs N moves per U steps.  After N steps the array M
// holds the inverse up to the pivot order: (P^{-1})_{k, p_j} = M_{p_k, j}.
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

template <int N, int NT, int U>
__global__ void __launch_bounds__(NT) k_gj_rows(double* __restrict__ blocks) {
  static_assert(N % U == 0, "whole groups of U steps");
  constexpr int NW = NT / 64;
  constexpr int CW = 4, PD = 3;  // pivot-row columns per LDS chunk, chunks read ahead
  static_assert(N % CW == 0, "whole chunks");
  __shared__ __align__(16) double rowp[N];   // the pivot row of the current step
  const double2* rp2 = reinterpret_cast<const double2*>(rowp);
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
  double rscale = 1.0;       // the row's pending factor 1/pivot

  for (int k0 = 0; k0 < N; k0 += U) {
#pragma unroll
    for (int c = 0; c < U; ++c) {
      // pivot: largest |a_{i,c}| over the candidate rows, ties to the lower row
      // (NaN entries never win the maximum; a wave whose candidates are all NaN still
      // offers its lowest candidate, a wave without candidates offers none)
      const bool cand = kstep < 0;
      const double mine = cand ? fabs(a[c]) : -1.0;
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
      const bool is_p = tid == p;
      if (is_p) {
#pragma unroll
        for (int j = 0; j < N; ++j) rowp[j] = a[j];
        kstep = k0 + c;
      }
      if (tid == 0) pivs[k0 + c] = p;
      __syncthreads();
      const double ipiv = 1.0 / rowp[c];
      // other rows: a_j <- a_j - (a_c / pivot) r_j, a_c <- -a_c / pivot;
      // the pivot row (g = 0) keeps its entries and takes a 1 in column c
      const double g = is_p ? 0.0 : a[c] * ipiv;
      if (is_p) rscale = ipiv;
      // the pivot row comes from LDS in chunks of CW columns, PD chunks ahead of the
      // FMAs that use it; the empty asm after a chunk's FMAs holds later reads back
      // (otherwise all N values are read into registers ahead of the FMAs)
      double2 buf[PD + 1][CW / 2];
#pragma unroll
      for (int q = 0; q < PD; ++q)
#pragma unroll
        for (int h = 0; h < CW / 2; ++h) buf[q][h] = rp2[q * (CW / 2) + h];
#pragma unroll
      for (int q = 0; q < N / CW; ++q) {
        if (q + PD < N / CW) {
#pragma unroll
          for (int h = 0; h < CW / 2; ++h) buf[(q + PD) % (PD + 1)][h] = rp2[(q + PD) * (CW / 2) + h];
        }
#pragma unroll
        for (int h = 0; h < CW / 2; ++h) {
          const int j = q * CW + 2 * h;
          if (j != c) a[j] = fma(-g, buf[q % (PD + 1)][h].x, a[j]);
          if (j + 1 != c) a[j + 1] = fma(-g, buf[q % (PD + 1)][h].y, a[j + 1]);
        }
        asm volatile("" : "+v"(a[q * CW]), "+v"(a[q * CW + 1]), "+v"(a[q * CW + 2]), "+v"(a[q * CW + 3]) : : "memory");
      }
      a[c] = is_p ? 1.0 : -g;
      // rowp is rewritten by the next step's pivot: with several waves the barrier of
      // the pivot search orders it, a single wave needs one here
      if (NW == 1) __syncthreads();
    }
    // rotate left by U: the next group's columns come to 0..U-1
    double t[U];
#pragma unroll
    for (int c = 0; c < U; ++c) t[c] = a[c];
#pragma unroll
    for (int j = 0; j < N - U; ++j) a[j] = a[j + U];
#pragma unroll
    for (int c = 0; c < U; ++c) a[N - U + c] = t[c];
  }
  // (P^{-1})_{k_r, p_j} = M_{r, j} / pivot_r: thread r writes row k_r of the inverse
  if (own && kstep >= 0 && kstep < N) {
#pragma unroll
    for (int j = 0; j < N; ++j) A[(size_t)min(max(pivs[j], 0), N - 1) * N + kstep] = a[j] * rscale;
  }
}

hipError_t launch_gj_rows_f64(int nb, double* blocks, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  // 36x36 and 64x64 blocks are inverted on the matrix cores (gj_mfma.hip)
  if (nb != 100) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_gj_rows<100, 128, 5>), dim3(nblk), dim3(128), 0, s, blocks);
  return hipGetLastError();
}

}  // namespace frjf
