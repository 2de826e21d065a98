// In-LDS Gauss-Jordan inversion with partial pivoting, shared by the Euler and
// Navier-Stokes element-Jacobi kernels.
#pragma once
#include <hip/hip_runtime.h>

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
