// In-LDS Gauss-Jordan inversion with partial pivoting, shared by the Euler and
// Navier-Stokes element-Jacobi kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace frjf {

// Gauss-Jordan inversion with partial pivoting of the LDS block A (column-major, leading dim LD).
template <typename T, int N, int LD, int NT>
__device__ void gj_invert(T* A, T* sf, int* piv_row, int* perm) {
  const int tid = threadIdx.x;
  __shared__ T red_v[NT / 64];
  __shared__ int red_i[NT / 64];
  for (int k = 0; k < N; ++k) {
    // pivot search over rows k..N-1 of column k
    T best = (T)-1;
    int bi = k;
    for (int i = k + tid; i < N; i += NT) {
      const T a = fabs(A[k * LD + i]);
      if (a > best) {
        best = a;
        bi = i;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const T ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if ((tid & 63) == 0) {
      red_v[tid >> 6] = best;
      red_i[tid >> 6] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      T b = red_v[0];
      int ii = red_i[0];
      for (int w = 1; w < NT / 64; ++w)
        if (red_v[w] > b || (red_v[w] == b && red_i[w] < ii)) {
          b = red_v[w];
          ii = red_i[w];
        }
      *piv_row = ii;
      perm[k] = ii;
    }
    __syncthreads();
    const int p = *piv_row;
    if (p != k)
      for (int j = tid; j < N; j += NT) {
        const T t = A[j * LD + k];
        A[j * LD + k] = A[j * LD + p];
        A[j * LD + p] = t;
      }
    __syncthreads();
    const T pv = A[k * LD + k];
    for (int i = tid; i < N; i += NT) sf[i] = A[k * LD + i];
    __syncthreads();
    const T ipv = (T)1 / pv;
    for (int j = tid; j < N; j += NT) A[j * LD + k] = (j == k ? (T)1 : A[j * LD + k]) * ipv;
    __syncthreads();
    for (int i = tid; i < N; i += NT) {
      if (i == k) continue;
      const T fi = sf[i];
      for (int j = 0; j < N; ++j) {
        const T akj = A[j * LD + k];
        const T aij = (j == k) ? (T)0 : A[j * LD + i];
        A[j * LD + i] = aij - fi * akj;
      }
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last first
  for (int k = N - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k)
      for (int i = tid; i < N; i += NT) {
        const T t = A[k * LD + i];
        A[k * LD + i] = A[p * LD + i];
        A[p * LD + i] = t;
      }
    __syncthreads();
  }
}

}  // namespace frjf

namespace frjf {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Blocked Gauss-Jordan inversion with partial pivoting of an NP x NP FP32 block in
// LDS (column-major, leading dimension LD, NP a multiple of 16, padding rows and
// columns set to the identity by the caller).  Panels of 16 columns are
// eliminated column by column (row swaps applied to whole rows at once); the
// deferred transformation of every column outside the panel is the rank-16
// product  A[:, out] <- A[:, out] + A[:, panel] X,  with the panel's own rows
// replaced by A11 X (X = the panel rows of A[:, out] before the update), run on
// v_mfma_f32_16x16x4f32 with FP32 accumulation.
// Scratch: X (16 * NP floats), cn (NP), rowc (16), perm (NP), piv_row.
template <int NP, int LD, int NT>
__device__ void gj_invert_mfma_f32(float* A, float* X, float* cn, float* rowc, int* perm, int* piv_row) {
  static_assert(NP % 16 == 0, "panel width 16");
  constexpr int NW = NT / 64;
  constexpr int NTILE = NP / 16;
  __shared__ float red_v[NW];
  __shared__ int red_i[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int k0 = 0; k0 < NP; k0 += 16) {
    // ---- panel: unblocked Gauss-Jordan restricted to columns k0..k0+15
    for (int c = k0; c < k0 + 16; ++c) {
      float best = -1.0f;
      int bi = c;
      for (int i = c + tid; i < NP; i += NT) {
        const float a = fabsf(A[c * LD + i]);
        if (a > best) {
          best = a;
          bi = i;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const float ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (lane == 0) {
        red_v[wave] = best;
        red_i[wave] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        float b = red_v[0];
        int ii = red_i[0];
        for (int w = 1; w < NW; ++w)
          if (red_v[w] > b || (red_v[w] == b && red_i[w] < ii)) {
            b = red_v[w];
            ii = red_i[w];
          }
        *piv_row = ii;
        perm[c] = ii;
      }
      __syncthreads();
      const int p = *piv_row;
      if (p != c)
        for (int j = tid; j < NP; j += NT) {
          const float t = A[j * LD + c];
          A[j * LD + c] = A[j * LD + p];
          A[j * LD + p] = t;
        }
      __syncthreads();
      const float ia = 1.0f / A[c * LD + c];
      for (int r = tid; r < NP; r += NT) cn[r] = (r == c) ? ia : -A[c * LD + r] * ia;
      if (tid < 16) rowc[tid] = A[(k0 + tid) * LD + c];
      __syncthreads();
      for (int idx = tid; idx < NP * 16; idx += NT) {
        const int r = idx % NP, jj = k0 + idx / NP;
        if (jj == c) continue;
        const float rc = rowc[jj - k0];
        A[jj * LD + r] = (r == c) ? cn[c] * rc : fmaf(cn[r], rc, A[jj * LD + r]);
      }
      for (int r = tid; r < NP; r += NT) A[c * LD + r] = cn[r];
      __syncthreads();
    }
    // ---- deferred rank-16 update of the other columns on MFMA
    for (int idx = tid; idx < 16 * NP; idx += NT) {
      const int i = idx / NP, j = idx % NP;
      X[idx] = A[j * LD + k0 + i];  // X[i][j]: panel row k0+i, column j
    }
    __syncthreads();
    const int pt = k0 / 16;
    for (int tile = wave; tile < NTILE * NTILE; tile += NW) {
      const int rt = tile % NTILE, ct = tile / NTILE;
      if (ct == pt) continue;
      f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int kcol = 4 * kk + (lane >> 4);
        const float a = A[(k0 + kcol) * LD + rt * 16 + (lane & 15)];
        const float b = X[kcol * NP + ct * 16 + (lane & 15)];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
      }
      const int col = ct * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt * 16 + 4 * (lane >> 4) + r;
        const bool panel_row = (row >= k0 && row < k0 + 16);
        A[col * LD + row] = (panel_row ? 0.0f : A[col * LD + row]) + acc[r];
      }
    }
    __syncthreads();
  }
  for (int k = NP - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k)
      for (int i = tid; i < NP; i += NT) {
        const float t = A[k * LD + i];
        A[k * LD + i] = A[p * LD + i];
        A[p * LD + i] = t;
      }
    __syncthreads();
  }
}

}  // namespace frjf

namespace frjf {

// LDS block geometry per precision: FP32 blocks are padded to a multiple of 16
// (identity in the padding) for the MFMA panel updates.
template <int Nb, typename T>
struct BlockLds {
  static constexpr bool mfma = std::is_same<T, float>::value;
  static constexpr int NP = mfma ? ((Nb + 15) / 16) * 16 : Nb;
  static constexpr int LD = NP + 1;
};

// Invert the block held in LDS (FP64: scalar Gauss-Jordan; FP32: blocked on MFMA).
template <typename T, int Nb, int NT>
__device__ void invert_lds(T* A, T* sf, int* piv_row, int* perm, float* X, float* rowc) {
  using L = BlockLds<Nb, T>;
  if constexpr (L::mfma) {
    const int tid = threadIdx.x;
    for (int idx = tid; idx < L::NP * L::NP; idx += NT) {
      const int c = idx / L::NP, r = idx % L::NP;
      if (c >= Nb || r >= Nb) A[c * L::LD + r] = (r == c) ? 1.0f : 0.0f;
    }
    __syncthreads();
    gj_invert_mfma_f32<L::NP, L::LD, NT>(reinterpret_cast<float*>(A), X, reinterpret_cast<float*>(sf), rowc, perm,
                                         piv_row);
  } else {
    gj_invert<T, Nb, L::LD, NT>(A, sf, piv_row, perm);
  }
}

}  // namespace frjf
