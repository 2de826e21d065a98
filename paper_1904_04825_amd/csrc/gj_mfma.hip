// Batched in-place inversion of the FP32 element-Jacobi blocks (Section 4.5) on
// the matrix cores.
//
// One wavefront per block.  The block, padded to NP = 16T with the identity, is
// held in registers as T x T tiles in the accumulator layout of
// v_mfma_f32_16x16x4f32: lane l = n + 16g holds column n of a tile and four of
// its rows.  Rows are labelled so that register r of lane group g is row
// g + 4r of the tile; with that labelling a tile's registers can be used as the
// B operand of the same instruction without moving data.
//
// Gauss-Jordan elimination with partial pivoting, blocked by panels of 16
// columns, as Jordan exchanges (no rows are moved; the pivot of a column is the
// largest candidate among the rows not pivoted yet):
//   panel K: the 16 exchanges restricted to tile column K (kept in tile column 0
//     by rotating the tile columns).  The pivot row's values reach every lane by one permute, the
//     pivot column's values reach the lanes of each 16-lane row by a DPP row
//     broadcast;
//   the other columns then take the 16 exchanges at once as a rank-16 product:
//     A[:, j] <- A[:, j] (pivot rows zeroed) + W A_P[j],  W = the transformed
//     panel, A_P[j] = the pivot rows of column j before the update,
//   with W and A_P staged through LDS into MFMA operand layout and FP32
//   accumulation on the matrix cores.
// After T panels the registers hold the inverse up to the pivot order:
// (P^{-1})_{k_i, p_j} = M_{i, j}, k_i the step that pivoted row i and p_j the
// row pivoted in step j.
#include "internal.h"

namespace frjf {

typedef float f32x4_t __attribute__((ext_vector_type(4)));

// One tile column: tile rt's four registers are entries 4 rt .. 4 rt + 3.  A
// uniform index into it compiles to an indexed register move.
template <int T>
struct ColT {
  typedef float type __attribute__((ext_vector_type(4 * T)));
};

template <int T>
__device__ __forceinline__ f32x4_t tile_of(const typename ColT<T>::type& c, int rt) {
  return f32x4_t{c[4 * rt], c[4 * rt + 1], c[4 * rt + 2], c[4 * rt + 3]};
}

// x from the lane 16 (XOR16) or 32 lanes away (lane l ^ 16, l ^ 32), by the row
// swap instructions (no LDS round trip)
__device__ __forceinline__ unsigned lane_xor16(unsigned x) {
  const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
  return ((threadIdx.x >> 4) & 1) ? r[0] : r[1];
}
__device__ __forceinline__ unsigned lane_xor32(unsigned x) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  return ((threadIdx.x >> 5) & 1) ? r[0] : r[1];
}
__device__ __forceinline__ float lane_xor16f(float x) { return __uint_as_float(lane_xor16(__float_as_uint(x))); }
__device__ __forceinline__ float lane_xor32f(float x) { return __uint_as_float(lane_xor32(__float_as_uint(x))); }

// x broadcast from lane C of each 16-lane row
template <int C>
__device__ __forceinline__ float row_bcast(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x), 0x150 + C, 0xf, 0xf, false));
}

template <int NP>
struct GjMfmaLds {
  float W[NP][17];       // transformed panel, [row][panel column]
  float B[16][NP + 4];   // pivot rows of the other columns, [pivot][column]
  int kstep[NP];         // step that pivoted each row
  int pstep[NP];         // row pivoted in each step
};

// One elimination step on the panel copy W (panel column C, global step s).
template <int T, int C>
__device__ __forceinline__ void panel_step(typename ColT<T>::type& W, unsigned& used, int s, int n, int g,
                                           GjMfmaLds<16 * T>& L) {
  // pivot: largest |a| of column C among the rows not pivoted yet.  Each entry
  // becomes one 32-bit key, the bits of |a| (monotone for non-negative floats)
  // with the low 7 mantissa bits replaced by 127 - (32 g + 4 rt + r): the unsigned
  // maximum picks the largest entry (entries within 2^-16 of each other count as
  // equal, the lower row code winning) and always decodes to a candidate row.
  // The four lanes of column C combine their maxima.
  unsigned key = 0u;
#pragma unroll
  for (int rt = 0; rt < T; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const unsigned k = (__float_as_uint(W[4 * rt + r]) & 0x7fffff80u) | (127u - (32u * g + 4u * rt + r));
      key = max(key, ((used >> (4 * rt + r)) & 1u) ? 0u : k);
    }
  key = max(key, lane_xor16(key));
  key = max(key, lane_xor32(key));
  const unsigned code = 127u - ((unsigned)__builtin_amdgcn_readlane((int)key, C) & 127u);
  const int p = min(16 * (int)((code & 31u) >> 2) + (int)(code >> 5) + 4 * (int)(code & 3u), 16 * T - 1);
  const int rtp = p >> 4, gp = (p & 15) & 3, rp = (p & 15) >> 2;
  const int idx = 4 * rtp + rp;
  if (g == gp) used |= 1u << idx;
  if (n == 0 && g == 0) {
    L.kstep[p] = s;
    L.pstep[s] = p;
  }
  // pivot row value of this lane's column, and the pivot
  // row p lives in lane group gp: lane (n, g) takes it from lane (n, gp)
  const float own = W[idx];
  const float o16 = lane_xor16f(own), o32 = lane_xor32f(own), o48 = lane_xor16f(o32);
  const int d = g ^ gp;
  const float pr = d == 0 ? own : (d == 1 ? o16 : (d == 2 ? o32 : o48));
  const float piv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pr), C));
  const float ipiv = 1.0f / piv;
  const float t = pr * ipiv;
  const bool colC = n == C;
  // other rows: a_ij -= a_iC a_pj / pivot; column C: -a_iC / pivot; row p: a_pj / pivot, 1/pivot
#pragma unroll
  for (int rt = 0; rt < T; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float f = row_bcast<C>(W[4 * rt + r]);
      const float u = fmaf(-f, t, W[4 * rt + r]);
      W[4 * rt + r] = colC ? -f * ipiv : u;
    }
  const float wp = W[idx];
  W[idx] = (g == gp) ? (colC ? ipiv : t) : wp;
}

template <int T, int C = 0>
__device__ __forceinline__ void panel_steps(typename ColT<T>::type& W, unsigned& used, int K, int n, int g,
                                            GjMfmaLds<16 * T>& L) {
  if constexpr (C < 16) {
    panel_step<T, C>(W, used, 16 * K + C, n, g, L);
    panel_steps<T, C + 1>(W, used, K, n, g, L);
  }
}

template <int T, int N>
__global__ void __launch_bounds__(64) k_gj_mfma(float* __restrict__ blocks) {
  constexpr int NP = 16 * T;
  __shared__ GjMfmaLds<NP> L;
  const int l = threadIdx.x, n = l & 15, g = l >> 4;
  float* A = blocks + (size_t)blockIdx.x * N * N;

  // block M[ct][4 rt + r]: lane (n, g) holds entry (16 rt + g + 4 r, 16 ct + n); identity padding
  typename ColT<T>::type M[T];
#pragma unroll
  for (int ct = 0; ct < T; ++ct)
#pragma unroll
    for (int rt = 0; rt < T; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * rt + g + 4 * r, j = 16 * ct + n;
        M[ct][4 * rt + r] = (i < N && j < N) ? A[(size_t)j * N + i] : (i == j ? 1.0f : 0.0f);
      }
  unsigned used = 0;  // bit 4 rt + r: row 16 rt + g + 4 r is pivoted
  for (int i = l; i < NP; i += 64) L.kstep[i] = -1;
  __syncthreads();

  // Panel K is always tile column 0: the tile columns rotate left by one after
  // every panel, so after T panels they are back in place.
  for (int K = 0; K < T; ++K) {
    // ---- panel: the 16 exchanges on tile column 0
    panel_steps<T>(M[0], used, K, n, g, L);

    // ---- stage W and the pivot rows of the other columns in LDS; zero those rows
#pragma unroll
    for (int rt = 0; rt < T; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) L.W[16 * rt + g + 4 * r][n] = M[0][4 * rt + r];
    __syncthreads();  // kstep of this panel's pivots
#pragma unroll
    for (int rt = 0; rt < T; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = L.kstep[16 * rt + g + 4 * r] - 16 * K;  // panel step that pivoted the row, if any
        const bool pivot_row = (unsigned)c < 16u;
#pragma unroll
        for (int ct = 1; ct < T; ++ct) {
          const float v = M[ct][4 * rt + r];
          if (pivot_row) L.B[c][16 * ct + n] = v;
          M[ct][4 * rt + r] = pivot_row ? 0.0f : v;
        }
      }
    __syncthreads();

    // ---- rank-16 update of the other tile columns on the matrix cores.  K index of
    // slice kk, lane group j: panel column 4 kk + j.  A operand: row m = n of the
    // output tile, i.e. row 16 rt + m/4 + 4 (m % 4) under the register labelling.
    float Wa[T][4];
#pragma unroll
    for (int rt = 0; rt < T; ++rt)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) Wa[rt][kk] = L.W[16 * rt + (n >> 2) + 4 * (n & 3)][4 * kk + g];
#pragma unroll
    for (int ct = 1; ct < T; ++ct) {
      float Bp[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) Bp[kk] = L.B[4 * kk + g][16 * ct + n];
#pragma unroll
      for (int rt = 0; rt < T; ++rt) {
        f32x4_t acc = tile_of<T>(M[ct], rt);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Wa[rt][kk], Bp[kk], acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) M[ct][4 * rt + r] = acc[r];
      }
    }
    // ---- rotate the tile columns left by one
    {
      const typename ColT<T>::type first = M[0];
#pragma unroll
      for (int ct = 0; ct + 1 < T; ++ct) M[ct] = M[ct + 1];
      M[T - 1] = first;
    }
    __syncthreads();  // LDS staging is reused by the next panel
  }

  // ---- (P^{-1})_{k_i, p_j} = M_{i, j}, column-major, the padding dropped
#pragma unroll
  for (int ct = 0; ct < T; ++ct)
#pragma unroll
    for (int rt = 0; rt < T; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * rt + g + 4 * r, j = 16 * ct + n;
        const int ki = L.kstep[i], pj = L.pstep[j];
        if (ki >= 0 && ki < N && pj >= 0 && pj < N) A[(size_t)pj * N + ki] = M[ct][4 * rt + r];
      }
}

hipError_t launch_gj_mfma_f32(int nb, float* blocks, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  switch (nb) {
    case 36:
      hipLaunchKernelGGL((k_gj_mfma<3, 36>), dim3(nblk), dim3(64), 0, s, blocks);
      break;
    case 64:
      hipLaunchKernelGGL((k_gj_mfma<4, 64>), dim3(nblk), dim3(64), 0, s, blocks);
      break;
    case 100:
      hipLaunchKernelGGL((k_gj_mfma<7, 100>), dim3(nblk), dim3(64), 0, s, blocks);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace frjf
