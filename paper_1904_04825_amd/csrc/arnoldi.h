// The Givens least-squares update of an Arnoldi step (Section 4.5, GMRES) as device
// code: run by a stand-alone kernel after the last step of a restart cycle and, for
// the other steps, by workgroup 0 of the next step's preconditioner kernel, which
// needs the same ||w|| to normalise the next basis vector.
#pragma once

#include "internal.h"
#include "wavesum.h"

namespace frjf {

struct GivensLds {
  double col[kMaxM + 2], cs[kMaxM], sn[kMaxM];
  double red[kRedThreads / 64];
};

// Sum of nb <= kRedThreads partial sums p[0 .. nb) over a workgroup of kRedThreads
// threads in one fixed order, returned to every thread (contains barriers).
__device__ __forceinline__ double block_sum_partials(const double* __restrict__ p, int nb, double* red) {
  const int tid = threadIdx.x;
  double s = wave_sum(tid < nb ? p[tid] : 0.0);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kRedThreads / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// Step j = st->j: the Hessenberg column h1 + h2 with h_{j+1,j} = sqrt(hn2) = ||w||,
// the earlier rotations applied to it, the new rotation, the least-squares residual
// |g_{j+1}| and the stop decision (converged, breakdown or NaN); the status block is
// also written to mapped host memory for the host's poll.  Every thread of the
// workgroup calls it.
__device__ __forceinline__ void givens_step(GmState* st, double hn2, int M, GivensLds& L) {
  const int tid = threadIdx.x;
  const int j = st->j;
  const int ld = M + 1;
  if (tid <= j) L.col[tid] = st->h1[tid] + st->h2[tid];
  if (tid < j) {
    L.cs[tid] = st->cs[tid];
    L.sn[tid] = st->sn[tid];
  }
  __syncthreads();
  if (tid == 0) {
    double* col = L.col;
    const double hn = sqrt(hn2);
    double w02 = hn2;  // ||w||^2 before orthogonalisation (Pythagoras)
    for (int i = 0; i <= j; ++i) w02 += col[i] * col[i];
    st->w0 = sqrt(w02);
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      const double t = L.cs[i] * col[i] + L.sn[i] * col[i + 1];
      col[i + 1] = -L.sn[i] * col[i] + L.cs[i] * col[i + 1];
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
  if (tid <= j + 1) st->H[(size_t)j * ld + tid] = L.col[tid];
}

}  // namespace frjf
