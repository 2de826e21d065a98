// The Givens least-squares update of an Arnoldi step (Section 4.5, GMRES) as device
// code, shared by the kernels that finish a Hessenberg column:
//   CGS2 (restarts longer than 32): the column of step j is final after the step;
//     the next step's preconditioner kernel rotates it in workgroup 0 (it needs the
//     same ||w|| to normalise the next basis vector), a stand-alone kernel after the
//     cycle's last step;
//   DCGS2 (delayed re-orthogonalisation): the column of step j is first-pass only and
//     becomes final in the second pass of step j + 1, which rotates it in workgroup 0;
//     breakdown is caught by the next preconditioner kernel, and a stand-alone kernel
//     rotates the cycle's last column as it stands.
#pragma once

#include "internal.h"
#include "wavesum.h"

namespace frjf {

struct GivensLds {
  double col[kMaxM + 2], cs[kMaxM], sn[kMaxM];
  double red[kRedThreads / 64];
};

// Sum of nb <= kRedBlocks partial sums p[0 .. nb) over a workgroup of kRedThreads
// threads in one fixed order, returned to every thread (contains barriers).
__device__ __forceinline__ double block_sum_partials(const double* __restrict__ p, int nb, double* red) {
  const int tid = threadIdx.x;
  double s = tid < nb ? p[tid] : 0.0;
  for (int b = tid + kRedThreads; b < nb; b += kRedThreads) s += p[b];
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kRedThreads / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// One thread: column k of the Hessenberg matrix, final, in col[0 .. k+1] (col[k+1] =
// h_{k+1,k}); cs, sn hold rotations 0 .. k-1.  Applies those rotations, forms rotation
// k, updates g, the least-squares residual |g_{k+1}| and the stop decision (NaN,
// converged, or breakdown when h_{k+1,k} <= 1e-14 w0, w0 = ||A z_k|| before
// orthogonalisation), sets st->j = k + 1 and copies the status block to mapped host
// memory.  The rotated column is left in col.
__device__ __forceinline__ void givens_rotate(GmState* st, int k, double* col, const double* cs, const double* sn,
                                              double w0) {
  const double hn = col[k + 1];
  for (int i = 0; i < k; ++i) {
    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  const double den = hypot(col[k], col[k + 1]);
  st->cs[k] = col[k] / den;
  st->sn[k] = col[k + 1] / den;
  col[k] = den;
  col[k + 1] = 0.0;
  st->g[k + 1] = -st->sn[k] * st->g[k];
  st->g[k] = st->cs[k] * st->g[k];
  const double rest = fabs(st->g[k + 1]);
  st->rest = rest;
  st->hn = hn;
  st->w0 = w0;
  st->j = k + 1;
  if (!(rest == rest) || !(den == den) || isinf(rest) || den == 0.0) {
    st->stop = 1;
    st->why = 3;
    st->done = 1;
  } else if (rest <= st->target) {
    st->stop = 1;
    st->why = 1;
    st->done = 1;
  } else if (!(hn > 1e-14 * w0)) {
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
    hs->evals = st->evals;
  }
}

// Loads rotations 0 .. k-1 into L (all threads; a barrier follows before use).
__device__ __forceinline__ void load_rotations(const GmState* st, int k, GivensLds& L) {
  const int tid = threadIdx.x;
  if (tid < k) {
    L.cs[tid] = st->cs[tid];
    L.sn[tid] = st->sn[tid];
  }
}

// Stores the rotated column k from L.col into H (all threads, after a barrier).
__device__ __forceinline__ void store_column(GmState* st, int k, int M, const GivensLds& L) {
  const int tid = threadIdx.x;
  if (tid <= k + 1) st->H[(size_t)k * (M + 1) + tid] = L.col[tid];
}

// CGS2, step j = st->j: the column h1 + h2 with h_{j+1,j} = sqrt(hn2) = ||w||, rotated
// (w0 by Pythagoras: ||w||^2 before orthogonalisation = hn2 + sum of the column's
// squares).  Every thread of the workgroup calls it.
__device__ __forceinline__ void givens_step(GmState* st, double hn2, int M, GivensLds& L) {
  const int tid = threadIdx.x;
  const int j = st->j;
  if (tid <= j) L.col[tid] = st->h1[tid] + st->h2[tid];
  load_rotations(st, j, L);
  __syncthreads();
  if (tid == 0) {
    double w02 = hn2;
    for (int i = 0; i <= j; ++i) w02 += L.col[i] * L.col[i];
    L.col[j + 1] = sqrt(hn2);
    givens_rotate(st, j, L.col, L.cs, L.sn, sqrt(w02));
  }
  __syncthreads();
  store_column(st, j, M, L);
}

// DCGS2: the first-pass column k = st->j (h1[0 .. k], h_{k+1,k} = hn) taken as it
// stands and rotated, with w0 = st->w0 (the cycle's last column, or a column whose
// next basis vector broke down).  Every thread of the workgroup calls it.
__device__ __forceinline__ void givens_first_pass(GmState* st, double hn, int M, GivensLds& L) {
  const int tid = threadIdx.x;
  const int k = st->j;
  if (tid <= k) L.col[tid] = st->h1[tid];
  load_rotations(st, k, L);
  __syncthreads();
  if (tid == 0) {
    L.col[k + 1] = hn;
    givens_rotate(st, k, L.col, L.cs, L.sn, st->w0);
  }
  __syncthreads();
  store_column(st, k, M, L);
}

}  // namespace frjf
