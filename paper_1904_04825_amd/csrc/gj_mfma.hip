// Batched in-place inversion of the element-Jacobi blocks (Section 4.5) on the
// matrix cores, FP32 (v_mfma_f32_16x16x4f32) and FP64 (v_mfma_f64_16x16x4f64).
//
// One wavefront per block.  The block, padded to NP = 16T with the identity, is
// held in registers as T x T tiles in the accumulator layout of the 16x16x4
// instruction: lane l = n + 16g holds column n of a tile and four of its rows,
// register r holding row g + 4r.  That is the FP64 instruction's own row order; the
// FP32 instruction keeps row 4g + r there, so for FP32 the rows are relabelled and
// the A operand takes its rows in the same relabelled order.
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
//   with W and A_P staged through LDS into MFMA operand layout and accumulation in
//   the block's precision on the matrix cores.
// After T panels the registers hold the inverse up to the pivot order:
// (P^{-1})_{k_i, p_j} = M_{i, j}, k_i the step that pivoted row i and p_j the
// row pivoted in step j.
#include "internal.h"

namespace frjf {

// One tile column: tile rt's four registers are entries 4 rt .. 4 rt + 3.  A
// uniform index into it compiles to an indexed register move.
template <typename S, int T>
struct ColT {
  typedef S type __attribute__((ext_vector_type(4 * T)));
};

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

// x broadcast from lane C of each 16-lane row (every lane has a source, so no
// old value is kept: the move needs no copy of x)
template <int C>
__device__ __forceinline__ unsigned row_bcast_u(unsigned x) {
  return (unsigned)__builtin_amdgcn_mov_dpp((int)x, 0x150 + C, 0xf, 0xf, true);
}

// The lane operations and the matrix instruction for one precision.  key_bits: 32
// bits whose unsigned order is the order of |x| (the high word for FP64).
template <typename S>
struct GjOps;
template <>
struct GjOps<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  // tile row held by A-operand lane row m (the accumulator keeps row 4g + r in
  // register r of lane group g, labelled g + 4r)
  __device__ static int a_row(int m) { return (m >> 2) + 4 * (m & 3); }
  __device__ static unsigned key_bits(float x) { return __float_as_uint(x); }
  __device__ static float xor16(float x) { return __uint_as_float(lane_xor16(__float_as_uint(x))); }
  __device__ static float xor32(float x) { return __uint_as_float(lane_xor32(__float_as_uint(x))); }
  template <int C>
  __device__ static float bcast(float x) { return __uint_as_float(row_bcast_u<C>(__float_as_uint(x))); }
  template <int C>
  __device__ static float readlane(float x) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), C)); }
  __device__ static v4 mfma(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <>
struct GjOps<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  // the accumulator keeps row g + 4r in register r of lane group g
  __device__ static int a_row(int m) { return m; }
  __device__ static unsigned lo(double x) { return (unsigned)__double2loint(x); }
  __device__ static unsigned hi(double x) { return (unsigned)__double2hiint(x); }
  __device__ static double mk(unsigned h, unsigned l) { return __hiloint2double((int)h, (int)l); }
  __device__ static unsigned key_bits(double x) { return hi(x); }
  __device__ static double xor16(double x) { return mk(lane_xor16(hi(x)), lane_xor16(lo(x))); }
  __device__ static double xor32(double x) { return mk(lane_xor32(hi(x)), lane_xor32(lo(x))); }
  template <int C>
  __device__ static double bcast(double x) { return mk(row_bcast_u<C>(hi(x)), row_bcast_u<C>(lo(x))); }
  template <int C>
  __device__ static double readlane(double x) {
    return mk((unsigned)__builtin_amdgcn_readlane((int)hi(x), C), (unsigned)__builtin_amdgcn_readlane((int)lo(x), C));
  }
  __device__ static v4 mfma(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};

template <typename S, int T>
__device__ __forceinline__ typename GjOps<S>::v4 tile_of(const typename ColT<S, T>::type& c, int rt) {
  return typename GjOps<S>::v4{c[4 * rt], c[4 * rt + 1], c[4 * rt + 2], c[4 * rt + 3]};
}

template <typename S, int NP>
struct GjMfmaLds {
  S W[NP][17];           // transformed panel, [row][panel column]
  S B[16][NP + 4];       // pivot rows of the other columns, [pivot][column]
  int kstep[NP];         // step that pivoted each row
  int pstep[NP];         // row pivoted in each step
};

// Per held row: the key mask 0x7fffff80 | (127 - (32 g + 4 rt + r)) while the row is
// a candidate, 0 once it is pivoted.
template <int T>
struct KeyMask {
  typedef unsigned type __attribute__((ext_vector_type(4 * T)));
};

// One elimination step on the panel copy W (panel column C, global step s).
template <typename S, int T, int C>
__device__ __forceinline__ void panel_step(typename ColT<S, T>::type& W, typename KeyMask<T>::type& km, int s, int n,
                                           int g, GjMfmaLds<S, 16 * T>& L) {
  using O = GjOps<S>;
  // pivot: largest |a| of column C among the rows not pivoted yet.  Each entry
  // becomes one 32-bit key, the bits of |a| (monotone for non-negative values; the
  // high word of an FP64 value) with the low 7 bits replaced by
  // 127 - (32 g + 4 rt + r): the unsigned maximum picks the largest entry (entries
  // within 2^-16 (FP32) or 2^-13 (FP64) of each other count as equal, the lower row
  // code winning) and always decodes to a candidate row.  The four lanes of column C
  // combine their maxima.  (bits | 127) & mask: the key of a candidate, 0 for a row
  // already pivoted.
  unsigned key = 0u;
#pragma unroll
  for (int e = 0; e < 4 * T; ++e) key = max(key, (O::key_bits(W[e]) | 127u) & km[e]);
  key = max(key, lane_xor16(key));
  key = max(key, lane_xor32(key));
  const unsigned code = 127u - ((unsigned)__builtin_amdgcn_readlane((int)key, C) & 127u);
  const int p = min(16 * (int)((code & 31u) >> 2) + (int)(code >> 5) + 4 * (int)(code & 3u), 16 * T - 1);
  const int rtp = p >> 4, gp = (p & 15) & 3, rp = (p & 15) >> 2;
  const int idx = 4 * rtp + rp;
  {
    // one indexed read and one indexed write (a conditional write would copy the vector)
    const unsigned cur = km[idx];
    km[idx] = (g == gp) ? 0u : cur;
  }
  if (n == 0 && g == 0) {
    L.kstep[p] = s;
    L.pstep[s] = p;
  }
  // pivot row value of this lane's column, and the pivot
  // row p lives in lane group gp: lane (n, g) takes it from lane (n, gp)
  const S own = W[idx];
  const S o16 = O::xor16(own), o32 = O::xor32(own), o48 = O::xor16(o32);
  const int d = g ^ gp;
  const S pr = d == 0 ? own : (d == 1 ? o16 : (d == 2 ? o32 : o48));
  const S piv = O::template readlane<C>(pr);
  const S ipiv = S(1) / piv;
  const S t = pr * ipiv;
  const bool colC = n == C;
  // other rows: a_ij -= a_iC a_pj / pivot; column C: -a_iC / pivot; row p: a_pj / pivot, 1/pivot.
  // One form for every lane, f (a_iC) + nt * (column C ? 0 : a_ij): on lane C, f is the
  // lane's own entry, so its new entry is f * (-1/pivot) exactly as a separate product
  // would round it
  const S nt = colC ? -ipiv : -t;
#pragma unroll
  for (int rt = 0; rt < T; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const S f = O::template bcast<C>(W[4 * rt + r]);
      const S ws = colC ? S(0) : W[4 * rt + r];
      W[4 * rt + r] = fma(f, nt, ws);
    }
  const S wp = W[idx];
  W[idx] = (g == gp) ? (colC ? ipiv : t) : wp;
}

template <typename S, int T, int C = 0>
__device__ __forceinline__ void panel_steps(typename ColT<S, T>::type& W, typename KeyMask<T>::type& km, int K, int n,
                                            int g,
                                            GjMfmaLds<S, 16 * T>& L) {
  if constexpr (C < 16) {
    panel_step<S, T, C>(W, km, 16 * K + C, n, g, L);
    panel_steps<S, T, C + 1>(W, km, K, n, g, L);
  }
}

// Waves per SIMD the register allocation aims at: FP64 with 4 x 4 tiles fits two
// in 206 VGPRs (left alone, the allocation takes 288 with accumulation registers and
// runs one wave per SIMD, 1.4x slower); the others keep the default.
template <typename S, int T>
struct GjWaves {
  static constexpr int value = (sizeof(S) == 8 && T == 4) ? 2 : 1;
};

template <typename S, int T, int N>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(GjWaves<S, T>::value)))
k_gj_mfma(S* __restrict__ blocks) {
  using O = GjOps<S>;
  constexpr int NP = 16 * T;
  __shared__ GjMfmaLds<S, NP> L;
  const int l = threadIdx.x, n = l & 15, g = l >> 4;
  S* A = blocks + (size_t)blockIdx.x * N * N;

  // block M[ct][4 rt + r]: lane (n, g) holds entry (16 rt + g + 4 r, 16 ct + n); identity padding
  typename ColT<S, T>::type M[T];
#pragma unroll
  for (int ct = 0; ct < T; ++ct)
#pragma unroll
    for (int rt = 0; rt < T; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * rt + g + 4 * r, j = 16 * ct + n;
        M[ct][4 * rt + r] = (i < N && j < N) ? A[(size_t)j * N + i] : (i == j ? S(1) : S(0));
      }
  typename KeyMask<T>::type km;  // entry 4 rt + r: row 16 rt + g + 4 r
#pragma unroll
  for (int rt = 0; rt < T; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) km[4 * rt + r] = 0x7fffff80u | (127u - (32u * g + 4u * rt + r));
  for (int i = l; i < NP; i += 64) L.kstep[i] = -1;
  __syncthreads();

  // Panel K is always tile column 0: the tile columns rotate left by one after
  // every panel, so after T panels they are back in place.
  for (int K = 0; K < T; ++K) {
    // ---- panel: the 16 exchanges on tile column 0
    panel_steps<S, T>(M[0], km, K, n, g, L);

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
          const S v = M[ct][4 * rt + r];
          if (pivot_row) L.B[c][16 * ct + n] = v;
          M[ct][4 * rt + r] = pivot_row ? S(0) : v;
        }
      }
    __syncthreads();

    // ---- rank-16 update of the other tile columns on the matrix cores.  K index of
    // slice kk, lane group j: panel column 4 kk + j.  A operand: instruction row m = n
    // of the output tile, i.e. tile row 16 rt + a_row(m).
    S Wa[T][4];
#pragma unroll
    for (int rt = 0; rt < T; ++rt)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) Wa[rt][kk] = L.W[16 * rt + O::a_row(n)][4 * kk + g];
#pragma unroll
    for (int ct = 1; ct < T; ++ct) {
      S Bp[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) Bp[kk] = L.B[4 * kk + g][16 * ct + n];
#pragma unroll
      for (int rt = 0; rt < T; ++rt) {
        typename O::v4 acc = tile_of<S, T>(M[ct], rt);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc = O::mfma(Wa[rt][kk], Bp[kk], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) M[ct][4 * rt + r] = acc[r];
      }
    }
    // ---- rotate the tile columns left by one
    {
      const typename ColT<S, T>::type first = M[0];
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
      hipLaunchKernelGGL((k_gj_mfma<float, 3, 36>), dim3(nblk), dim3(64), 0, s, blocks);
      break;
    case 64:
      hipLaunchKernelGGL((k_gj_mfma<float, 4, 64>), dim3(nblk), dim3(64), 0, s, blocks);
      break;
    case 100:
      hipLaunchKernelGGL((k_gj_mfma<float, 7, 100>), dim3(nblk), dim3(64), 0, s, blocks);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static hipError_t launch_gj_mfma_f64(int nb, double* blocks, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  switch (nb) {
    case 36:
      hipLaunchKernelGGL((k_gj_mfma<double, 3, 36>), dim3(nblk), dim3(64), 0, s, blocks);
      break;
    case 64:
      hipLaunchKernelGGL((k_gj_mfma<double, 4, 64>), dim3(nblk), dim3(64), 0, s, blocks);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// FP64 blocks of order 36 and 64 fit the registers of one wavefront (180 and 288
// VGPRs); order 100 (7 x 7 tiles of four FP64 values per lane) does not and stays on
// the row kernel.
hipError_t launch_invert_f64(int nb, double* blocks, int nblk, hipStream_t s) {
  if (nb == 36 || nb == 64) return launch_gj_mfma_f64(nb, blocks, nblk, s);
  if (nb == 144 || nb == 196) return launch_gj_wide_f64(nb, blocks, nblk, s);
  return launch_gj_rows_f64(nb, blocks, nblk, s);
}

hipError_t launch_invert_f32(int nb, float* blocks, int nblk, hipStream_t s) {
  if (nb == 144 || nb == 196) return launch_gj_wide_f32(nb, blocks, nblk, s);
  return launch_gj_mfma_f32(nb, blocks, nblk, s);
}

}  // namespace frjf
