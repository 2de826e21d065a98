// Implicit time steps on the 3D hexahedral FR path: the Jacobian-free linear solve of
// Section 4.5 and the ROW, ESDIRK and BDF2 steps of Sections 4.1-4.4 on the hexahedral
// discretisation (the Taylor-Green comparison of Section 5.3).
//
//   Element-Jacobi: blocks shift I - dR_e/dq_e of Nb = 5 (P+1)^3 rows (135 at P2, 320 at
//   P3).  Columns come from one-sided differences of the residual with every element of
//   one colour perturbed at once (colours chosen so that face neighbours differ, so each
//   such element sees unperturbed neighbours); only that colour's elements are
//   re-evaluated, eight columns per launch in separate copies of the state.  A 320 x 320
//   FP64 block fits neither a workgroup's registers nor its LDS, so the inversion is a
//   panel Gauss-Jordan, one thread per row, that keeps the panel's columns in registers
//   and streams the rest of the block through global memory once per panel.  Blocks and
//   inverses are column-major per element, FP64 or FP32 (the preconditioner's precision).
//   FGMRES(m): classical Gram-Schmidt applied twice; the Hessenberg column, the Givens
//   rotations and the stopping tests run on the host, one synchronisation per Arnoldi
//   step (a 3D residual costs far more than that round trip).
//   PTC, ROW, ESDIRK and BDF2 follow the 2D drivers step for step (same options and
//   statistics, no learned starts).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "internal.h"
#include "solvers.h"
#include "wavesum.h"

namespace frjf {

namespace {

constexpr int kVec3 = 12; // state-sized vectors of a step
constexpr int kCopies = 8; // block columns evaluated per launch in the assembly

#define FR3_TRY(expr)        \
  do {                       \
    fr_status st_ = (expr);  \
    if (st_ < 0) return st_; \
  } while (0)

// ---------------------------------------------------------------- colouring
__device__ __forceinline__ int colour_of(int e, int nx, int ny, int c) {
  const int ex = e % nx, ey = (e / nx) % ny, ez = e / (nx * ny);
  return (ex + ey + ez) % c;
}

// Copy c = blockIdx.y of the perturbed states (Up + c ndof, steps dl + c nel): restores
// entry prev0 + c (v * np + k; none if prev0 < 0 or out of range) from U for the elements
// of colour col, then moves entry next0 + c (none if next0 < 0 or out of range) by
// delta_e = 1e-8 max(1, |U|).
__global__ void k3a_perturb(double* __restrict__ Up, const double* __restrict__ U, double* __restrict__ dl,
                            int nel, int np, int prev0, int next0, int nx, int ny, int c, int col, size_t ndof) {
  const int cp = blockIdx.y, nb = 5 * np;
  const int prev = prev0 < 0 ? -1 : prev0 + cp, next = next0 < 0 ? -1 : next0 + cp;
  double* u = Up + cp * ndof;
  double* d = dl + (size_t)cp * nel;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nel; e += gridDim.x * blockDim.x) {
    if (colour_of(e, nx, ny, c) != col) continue;
    if (prev >= 0 && prev < nb) {
      const size_t i = ((size_t)(prev / np) * nel + e) * np + prev % np;
      u[i] = U[i];
    }
    if (next >= 0 && next < nb) {
      const size_t i = ((size_t)(next / np) * nel + e) * np + next % np;
      const double x = U[i];
      const double del = 1e-8 * fmax(1.0, fabs(x));
      d[e] = del;
      u[i] = x + del;
    }
  }
}

// Column j = j0 + blockIdx.y of the blocks of the elements of colour col, from copy
// blockIdx.y: -(Rp_e - R0_e) / delta_e, plus shift on the diagonal, rounded to T.
// B[e][j][row].
template <typename T>
__global__ void k3a_column(T* __restrict__ B, const double* __restrict__ Rp, const double* __restrict__ R0,
                           const double* __restrict__ dl, int nel, int np, int j0, double shift, int nx, int ny, int c,
                           int col, size_t ndof) {
  const int nb = 5 * np, cp = blockIdx.y, j = j0 + cp;
  if (j >= nb) return;
  const double* rp = Rp + cp * ndof;
  const double* d = dl + (size_t)cp * nel;
  const size_t total = (size_t)nel * nb;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int e = (int)(t / nb), r = (int)(t % nb);
    if (colour_of(e, nx, ny, c) != col) continue;
    const size_t i = ((size_t)(r / np) * nel + e) * np + r % np;
    double v = -(rp[i] - R0[i]) / d[e];
    if (r == j) v += shift;
    B[((size_t)e * nb + j) * nb + r] = (T)v;
  }
}

// ---------------------------------------------------------------- inversion
// In-place Gauss-Jordan of one N x N block per workgroup with partial pivoting by
// Jordan exchanges: no rows move; step k takes as pivot the row p_k with the largest
// |a| in column k among the rows not pivoted yet (ties to the lower row, NaN never
// wins; if every candidate is NaN, the lowest candidate row).  One thread per row.
// Panels of W columns (W divides N): each thread holds its row of the panel in
// registers, rotated so that the step's column is always the first (one rotation per
// step, W per panel, so the panel ends in its own order; the step loop then stays rolled:
// 2.5k instructions against 14.8k unrolled, at the same speed), the pivot row broadcast through
// LDS; every other column j then becomes (column j with the panel's pivot rows zeroed)
// + Panel * (column j's old entries at those rows), JB columns per barrier: each thread
// loads its row's entries, the pivot rows' threads publish theirs in LDS, and each thread
// forms its new entries from its panel row.  The block streams through global memory once
// per panel.  After all panels A^{-1}[k][p_j] = M[p_k][j]; the inverse goes column-major
// to out.  T = double, or float for the FP32 preconditioner (arithmetic in T).
template <int N, int W, typename T>
__global__ void __launch_bounds__((N + 63) / 64 * 64, 1) k3_gj(T* __restrict__ A, T* __restrict__ out) {
  static_assert(N % W == 0, "whole panels");
  constexpr int NT = (N + 63) / 64 * 64, NW = NT / 64, JB = 16;
  __shared__ T rowp[W];
  __shared__ T ap[W][JB];
  __shared__ int pv[N];
  __shared__ double wb[NW];
  __shared__ int wi[NW], wm[NW];
  const int i = threadIdx.x, lane = i & 63, wid = i >> 6;
  const bool own = i < N;
  T* a = A + (size_t)blockIdx.x * N * N;
  int kst = own ? -1 : N;  // step that pivoted this row; -1 while a candidate
  for (int c0 = 0; c0 < N; c0 += W) {
    T pr[W];
#pragma unroll
    for (int cc = 0; cc < W; ++cc) pr[cc] = own ? a[(size_t)(c0 + cc) * N + i] : T(0);
#pragma unroll 1
    for (int c = 0; c < W; ++c) {
      // the step's column is pr[0]
      const bool cand = own && kst < 0;
      const double v = fabs((double)pr[0]);
      double best = -1.0;
      int bi = N, mc = cand ? i : N;
      if (cand && v > best) {
        best = v;
        bi = i;
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off), om = __shfl_xor(mc, off);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
        mc = min(mc, om);
      }
      if (lane == 0) {
        wb[wid] = best;
        wi[wid] = bi;
        wm[wid] = mc;
      }
      __syncthreads();
      double b = wb[0];
      int p = wi[0], m = wm[0];
#pragma unroll
      for (int q = 1; q < NW; ++q) {
        if (wb[q] > b || (wb[q] == b && wi[q] < p)) {
          b = wb[q];
          p = wi[q];
        }
        m = min(m, wm[q]);
      }
      if (p >= N) p = m;  // every candidate entry NaN
      if (i == p) {
        kst = c0 + c;
        pv[c0 + c] = p;
#pragma unroll
        for (int cc = 0; cc < W; ++cc) rowp[cc] = pr[cc];
      }
      __syncthreads();
      const T ipiv = T(1) / rowp[0];
      if (own) {
        if (i == p) {
          pr[0] = ipiv;
#pragma unroll
          for (int cc = 1; cc < W; ++cc) pr[cc] = rowp[cc] * ipiv;
        } else {
          const T f = pr[0] * ipiv;
          pr[0] = -f;
#pragma unroll
          for (int cc = 1; cc < W; ++cc) pr[cc] = fma(-f, rowp[cc], pr[cc]);
        }
      }
      const T t0 = pr[0];  // rotate: the next step's column to the front
#pragma unroll
      for (int cc = 0; cc + 1 < W; ++cc) pr[cc] = pr[cc + 1];
      pr[W - 1] = t0;
    }
    if (own) {
#pragma unroll
      for (int cc = 0; cc < W; ++cc) a[(size_t)(c0 + cc) * N + i] = pr[cc];
    }
    // this panel's pivot slot of the row (-1: not one of its pivots)
    const int slot = (kst >= c0 && kst < c0 + W) ? kst - c0 : -1;
    for (int j0 = 0; j0 < N; j0 += JB) {
      T x[JB];
#pragma unroll
      for (int t = 0; t < JB; ++t) {
        const int j = j0 + t;
        const bool live = own && j < N && (j < c0 || j >= c0 + W);
        x[t] = live ? a[(size_t)j * N + i] : T(0);
      }
      if (slot >= 0) {
#pragma unroll
        for (int t = 0; t < JB; ++t) ap[slot][t] = x[t];
      }
      __syncthreads();
      if (own) {
#pragma unroll
        for (int t = 0; t < JB; ++t) {
          const int j = j0 + t;
          if (j >= N || (j >= c0 && j < c0 + W)) continue;
          T v = slot >= 0 ? T(0) : x[t];
#pragma unroll
          for (int cc = 0; cc < W; ++cc) v = fma(pr[cc], ap[cc][t], v);
          a[(size_t)j * N + i] = v;
        }
      }
      __syncthreads();
    }
  }
  T* o = out + (size_t)blockIdx.x * N * N;
  for (int j = wid; j < N; j += NW) {
    const T* col = a + (size_t)j * N;
    T* oc = o + (size_t)pv[j] * N;
    for (int k = lane; k < N; k += 64) oc[k] = col[pv[k]];
  }
}

// z_e = inv_e r_e, one workgroup per element, one thread per row; inv column-major, in T
// (r rounded to T, the sums in T).
template <int N, typename T>
__global__ void __launch_bounds__((N + 63) / 64 * 64) k3_ej_apply(const T* __restrict__ inv,
                                                                 const double* __restrict__ r,
                                                                 double* __restrict__ z, int nel, int np) {
  __shared__ T rs[N];
  const int e = blockIdx.x, i = threadIdx.x;
  if (i < N) rs[i] = (T)r[((size_t)(i / np) * nel + e) * np + i % np];
  __syncthreads();
  if (i >= N) return;
  const T* B = inv + (size_t)e * N * N + i;
  T acc[4] = {T(0), T(0), T(0), T(0)};
  int j = 0;
  for (; j + 4 <= N; j += 4) {
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = fma(B[(size_t)(j + q) * N], rs[j + q], acc[q]);
  }
  for (; j < N; ++j) acc[0] = fma(B[(size_t)j * N], rs[j], acc[0]);
  z[((size_t)(i / np) * nel + e) * np + i % np] = (double)((acc[0] + acc[1]) + (acc[2] + acc[3]));
}

// ---------------------------------------------------------------- Krylov helpers
// part[b * nv + i] = partial sum of V_i . w over block b's grid-stride share.
__global__ void __launch_bounds__(kRedThreads) k3_mdot(const double* __restrict__ V, int nv,
                                                     const double* __restrict__ w, size_t n,
                                                     double* __restrict__ part) {
  constexpr int CH = 8;
  __shared__ double red[CH][kRedThreads / 64];
  for (int i0 = 0; i0 < nv; i0 += CH) {
    double acc[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) acc[q] = 0.0;
    for (size_t t = blockIdx.x * (size_t)kRedThreads + threadIdx.x; t < n; t += (size_t)gridDim.x * kRedThreads) {
      const double wt = w[t];
#pragma unroll
      for (int q = 0; q < CH; ++q)
        if (i0 + q < nv) acc[q] = fma(V[(size_t)(i0 + q) * n + t], wt, acc[q]);
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) acc[q] = wave_sum(acc[q]);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
      for (int q = 0; q < CH; ++q) red[q][threadIdx.x >> 6] = acc[q];
    __syncthreads();
    if (threadIdx.x < CH && i0 + (int)threadIdx.x < nv) {
      double s = 0.0;
      for (int q = 0; q < kRedThreads / 64; ++q) s += red[threadIdx.x][q];
      part[(size_t)blockIdx.x * nv + i0 + threadIdx.x] = s;
    }
    __syncthreads();
  }
}

// y += sgn sum_{i < nv} c[i] X_i, the coefficients on the device.
__global__ void k3_maxpy(double* __restrict__ y, const double* __restrict__ X, int nv, const double* __restrict__ c,
                         double sgn, size_t n) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
    double v = y[t];
    for (int i = 0; i < nv; ++i) v = fma(sgn * c[i], X[(size_t)i * n + t], v);
    y[t] = v;
  }
}

unsigned grid_of(size_t n, unsigned cap) { return (unsigned)std::max<size_t>(1, std::min<size_t>((n + 255) / 256, cap)); }

// ---------------------------------------------------------------- workspace
size_t al(size_t b) { return (b + 255) & ~(size_t)255; }
size_t block_store(const fr3d_disc* d) {
  const size_t nb = 5 * (size_t)d->np;
  return sizeof(double) * (size_t)d->nel * nb * nb;
}
constexpr int kHost = 3 * (kMaxM + 1) + 8;  // device/host scalars of one Arnoldi step

struct W3 {
  double* traces;   // residual traces and gradients
  double* scal;     // ||v||^2 of the JF epsilon
  double* partials; // reduction partials
  double* blocks;   // assembled blocks (destroyed by the inversion)
  double* inv;      // the preconditioner (inverse blocks) of the step drivers
  double* dl;       // per-element finite-difference steps, kCopies x nel
  int* elist;       // the elements grouped by colour
  double* Up;       // perturbed states, kCopies x ndof
  double* Rp;       // their residuals, kCopies x ndof
  char* Tc;         // their face data, kCopies x fr3d_trace_bytes (256-aligned)
  double* V;        // m + 1 basis vectors
  double* Z;        // m preconditioned vectors
  double* w;
  double* r;
  double* hd;       // kHost doubles
  double* part;     // kRedBlocks * (kMaxM + 1) multi-dot partials
  double* vec[kVec3];
};

W3 carve(const fr3d_disc* d, void* work, int m) {
  const size_t n = d->ndof;
  char* p = (char*)work;
  auto take = [&](size_t b) {
    void* r = p;
    p += al(b);
    return (double*)r;
  };
  W3 w{};
  w.traces = take(fr3d_trace_bytes(d));
  w.scal = take(256);
  w.partials = take(sizeof(double) * std::max<size_t>(kRedBlocks, 5 * (size_t)d->nel));
  w.blocks = take(block_store(d));
  w.inv = take(block_store(d));
  w.dl = take(sizeof(double) * d->nel * kCopies);
  w.elist = (int*)take(sizeof(int) * d->nel);
  w.Up = take(sizeof(double) * n * kCopies);
  w.Rp = take(sizeof(double) * n * kCopies);
  w.Tc = (char*)take(al(fr3d_trace_bytes(d)) * kCopies);
  w.V = take(sizeof(double) * n * (size_t)(m + 1));
  w.Z = take(sizeof(double) * n * (size_t)m);
  w.w = take(sizeof(double) * n);
  w.r = take(sizeof(double) * n);
  w.hd = take(sizeof(double) * kHost);
  w.part = take(sizeof(double) * (size_t)kRedBlocks * (kMaxM + 1));
  for (int i = 0; i < kVec3; ++i) w.vec[i] = take(sizeof(double) * n);
  return w;
}

size_t carve_bytes(const fr3d_disc* d, int m) {
  const size_t n = d->ndof;
  return al(fr3d_trace_bytes(d)) + al(256) + al(sizeof(double) * std::max<size_t>(kRedBlocks, 5 * (size_t)d->nel)) +
         2 * al(block_store(d)) + al(sizeof(double) * d->nel * kCopies) + al(sizeof(int) * d->nel) +
         2 * al(sizeof(double) * n * kCopies) + al(al(fr3d_trace_bytes(d)) * kCopies) +
         al(sizeof(double) * n * (size_t)(m + 1)) + al(sizeof(double) * n * (size_t)m) + 2 * al(sizeof(double) * n) +
         al(sizeof(double) * kHost) + al(sizeof(double) * (size_t)kRedBlocks * (kMaxM + 1)) +
         kVec3 * al(sizeof(double) * n);
}

fr_status read_dev(void* host, const void* dev, size_t bytes, hipStream_t s) {
  FR_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
  FR_HIP(hipStreamSynchronize(s));
  return FR_OK;
}

fr_status lin(double* y, std::initializer_list<std::pair<const double*, double>> terms, size_t n, hipStream_t s) {
  const double* xs[8];
  double cs[8];
  int k = 0;
  for (auto& t : terms) {
    xs[k] = t.first;
    cs[k++] = t.second;
  }
  FR_HIP(launch_lincomb(y, k, xs, cs, n, s));
  return FR_OK;
}

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

fr_status residual(const fr3d_disc* d, const double* U, double* R, W3& W, hipStream_t s) {
  FR_HIP(launch_fr3d_residual(d, 0, U, nullptr, nullptr, 0.0, 0.0, FR_EPS_ABS, nullptr, R, W.traces, s));
  return FR_OK;
}

// ---------------------------------------------------------------- element-Jacobi
int colour_count(const fr3d_disc* d) {
  for (int c = 2;; ++c)
    if (d->nx % c != 1 && d->ny % c != 1 && d->nz % c != 1) return c;
}

// Blocks shift I - dR_e/dq_e at U into B (column-major per element); R0 = R(U).  Per
// colour, kCopies block columns at a time, each in its own copy of the state and face
// data: only that colour's elements are re-evaluated, their traces from the perturbed
// state, their residuals against the neighbours' face data at U (one full evaluation at U
// first, copied to every copy; each copy's colour data restored after the colour).
fr_status assemble(const fr3d_disc* d, const double* U, const double* R0, double shift, void* B, int prec, W3& W,
                   hipStream_t s) {
  const int nb = 5 * d->np, nc = colour_count(d);
  const size_t n = d->ndof, tb = al(fr3d_trace_bytes(d));
  const unsigned ge = grid_of((size_t)d->nel, 4096), gc = grid_of((size_t)d->nel * nb, 8192);
  std::vector<int> list;
  std::vector<int> off(nc + 1, 0);
  list.reserve(d->nel);
  for (int col = 0; col < nc; ++col) {
    for (int e = 0; e < d->nel; ++e) {
      const int ex = e % d->nx, ey = (e / d->nx) % d->ny, ez = e / (d->nx * d->ny);
      if ((ex + ey + ez) % nc == col) list.push_back(e);
    }
    off[col + 1] = (int)list.size();
  }
  FR_HIP(hipMemcpyAsync(W.elist, list.data(), sizeof(int) * list.size(), hipMemcpyHostToDevice, s));
  FR3_TRY(residual(d, U, W.Rp, W, s));  // every element's face data at U
  for (int c = 0; c < kCopies; ++c) {
    FR_HIP(hipMemcpyAsync(W.Tc + c * tb, W.traces, fr3d_trace_bytes(d), hipMemcpyDeviceToDevice, s));
    FR_HIP(hipMemcpyAsync(W.Up + c * n, U, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  }
  for (int col = 0; col < nc; ++col) {
    const int* el = W.elist + off[col];
    const int cnt = off[col + 1] - off[col];
    if (cnt == 0) continue;
    int last = -1;
    for (int j0 = 0; j0 < nb; j0 += kCopies) {
      const int k = std::min(kCopies, nb - j0);
      hipLaunchKernelGGL(k3a_perturb, dim3(ge, kCopies), dim3(256), 0, s, W.Up, U, W.dl, d->nel, d->np, last, j0,
                         d->nx, d->ny, nc, col, n);
      FR_HIP(hipGetLastError());
      FR_HIP(launch_fr3d_residual_subset(d, W.Up, W.Rp, W.Tc, el, cnt, k, tb, false, s));
      if (prec == FR_F32)
        hipLaunchKernelGGL(k3a_column<float>, dim3(gc, k), dim3(256), 0, s, (float*)B, W.Rp, R0, W.dl, d->nel,
                           d->np, j0, shift, d->nx, d->ny, nc, col, n);
      else
        hipLaunchKernelGGL(k3a_column<double>, dim3(gc, k), dim3(256), 0, s, (double*)B, W.Rp, R0, W.dl, d->nel,
                           d->np, j0, shift, d->nx, d->ny, nc, col, n);
      FR_HIP(hipGetLastError());
      last = j0;
    }
    hipLaunchKernelGGL(k3a_perturb, dim3(ge, kCopies), dim3(256), 0, s, W.Up, U, W.dl, d->nel, d->np, last, -1,
                       d->nx, d->ny, nc, col, n);
    FR_HIP(hipGetLastError());
    FR_HIP(launch_fr3d_residual_subset(d, W.Up, W.Rp, W.Tc, el, cnt, kCopies, tb, true, s));  // colour data at U
  }
  FR_HIP(hipStreamSynchronize(s));  // the element lists were copied from this frame
  return FR_OK;
}

template <typename T>
fr_status invert_t(const fr3d_disc* d, T* B, T* inv, hipStream_t s) {
  switch (d->p) {
    // panel widths that divide N (whole panels keep the panel row in registers)
    case 2: hipLaunchKernelGGL((k3_gj<135, 27, T>), dim3(d->nel), dim3(192), 0, s, B, inv); break;
    case 3: hipLaunchKernelGGL((k3_gj<320, 32, T>), dim3(d->nel), dim3(320), 0, s, B, inv); break;
    default: return set_error(FR_EINVAL, "3D element-Jacobi: p must be 2 or 3");
  }
  FR_HIP(hipGetLastError());
  return FR_OK;
}

fr_status invert(const fr3d_disc* d, void* B, void* inv, int prec, hipStream_t s) {
  return prec == FR_F32 ? invert_t(d, (float*)B, (float*)inv, s) : invert_t(d, (double*)B, (double*)inv, s);
}

template <typename T>
fr_status apply_t(const fr3d_disc* d, const T* inv, const double* r, double* z, hipStream_t s) {
  switch (d->p) {
    case 2: hipLaunchKernelGGL((k3_ej_apply<135, T>), dim3(d->nel), dim3(192), 0, s, inv, r, z, d->nel, d->np); break;
    case 3: hipLaunchKernelGGL((k3_ej_apply<320, T>), dim3(d->nel), dim3(320), 0, s, inv, r, z, d->nel, d->np); break;
    default: return set_error(FR_EINVAL, "3D element-Jacobi: p must be 2 or 3");
  }
  FR_HIP(hipGetLastError());
  return FR_OK;
}

fr_status apply(const fr3d_disc* d, const void* inv, int prec, const double* r, double* z, hipStream_t s) {
  return prec == FR_F32 ? apply_t(d, (const float*)inv, r, z, s) : apply_t(d, (const double*)inv, r, z, s);
}

// The step drivers' preconditioner at (U, R0 = R(U), shift) into W.inv.
fr_status factor(const fr3d_disc* d, const double* U, const double* R0, double shift, int prec, W3& W,
                 hipStream_t s) {
  FR3_TRY(assemble(d, U, R0, shift, W.blocks, prec, W, s));
  return invert(d, W.blocks, W.inv, prec, s);
}

// ---------------------------------------------------------------- FGMRES(m)
struct JfArgs {
  const double* U;
  const double* R0;
  double shift, eps;
  int eps_mode;
};

fr_status jf(const fr3d_disc* d, const JfArgs& a, const double* v, double* out, W3& W, long* evals, hipStream_t s) {
  if (a.eps_mode == FR_EPS_RMS) FR_HIP(launch_norm2(v, d->ndof, W.partials, W.scal, nullptr, s));
  FR_HIP(launch_fr3d_residual(d, 1, a.U, v, a.R0, a.shift, a.eps, a.eps_mode, W.scal, out, W.traces, s));
  ++*evals;
  return FR_OK;
}

fr_status norm(const fr3d_disc* d, const double* x, W3& W, double* host, hipStream_t s) {
  FR_HIP(launch_norm2(x, d->ndof, W.partials, W.hd + kHost - 1, nullptr, s));
  double v = 0.0;
  FR3_TRY(read_dev(&v, W.hd + kHost - 1, sizeof(double), s));
  *host = std::sqrt(v);
  return FR_OK;
}

// h[0 .. nv) = V^T w into W.hd + off, then w -= V h.
fr_status cgs_pass(const fr3d_disc* d, int nv, W3& W, int off, hipStream_t s) {
  const size_t n = d->ndof;
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(k3_mdot, dim3(nb), dim3(kRedThreads), 0, s, W.V, nv, W.w, n, W.part);
  FR_HIP(hipGetLastError());
  FR_HIP(launch_finalize(W.part, nb, nv, nv, W.hd + off, nullptr, s));
  hipLaunchKernelGGL(k3_maxpy, dim3(grid_of(n, 4096)), dim3(256), 0, s, W.w, W.V, nv, W.hd + off, -1.0, n);
  FR_HIP(hipGetLastError());
  return FR_OK;
}

fr_status gmres(const fr3d_disc* d, const void* inv, int prec, const JfArgs& a, const double* b, double* x, bool x_zero,
                const fr_gmres_opts& o, fr_gmres_stats* out, W3& W, hipStream_t s) {
  const size_t n = d->ndof;
  const int m = o.m;
  const int max_iters = o.max_iters > 0 ? o.max_iters : 50 * m;
  fr_gmres_stats S{};
  long evals = 0;
  double beta = 0.0;
  if (x_zero) {
    FR3_TRY(lin(W.r, {{b, 1.0}}, n, s));
  } else {
    FR3_TRY(jf(d, a, x, W.w, W, &evals, s));
    FR3_TRY(lin(W.r, {{b, 1.0}, {W.w, -1.0}}, n, s));
  }
  FR3_TRY(norm(d, W.r, W, &beta, s));
  S.r_ref = o.ref_norm > 0 ? o.ref_norm : beta;
  const double target = o.rtol * S.r_ref;
  S.r_final = beta;
  fr_status result = FR_NOTCONV;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), hh(kHost);
  if (!std::isfinite(beta)) {
    result = FR_ENAN;
  } else if (beta <= target) {
    S.converged = 1;
    result = FR_OK;
  }
  while (result == FR_NOTCONV) {
    FR3_TRY(lin(W.V, {{W.r, 1.0 / beta}}, n, s));
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    bool conv = false, bad = false;
    for (int j = 0; j < m; ++j) {
      double* vj = W.V + (size_t)j * n;
      double* zj = W.Z + (size_t)j * n;
      FR3_TRY(apply(d, inv, prec, vj, zj, s));
      FR3_TRY(jf(d, a, zj, W.w, W, &evals, s));
      FR_HIP(launch_norm2(W.w, n, W.partials, W.hd + 2 * (kMaxM + 1), nullptr, s));      // ||w||^2 before
      FR3_TRY(cgs_pass(d, j + 1, W, 0, s));
      FR3_TRY(cgs_pass(d, j + 1, W, kMaxM + 1, s));
      FR_HIP(launch_norm2(W.w, n, W.partials, W.hd + 2 * (kMaxM + 1) + 1, nullptr, s));  // ||w||^2 after
      FR3_TRY(read_dev(hh.data(), W.hd, sizeof(double) * (2 * (kMaxM + 1) + 2), s));
      double* col = H.data() + (size_t)j * (m + 1);
      for (int i = 0; i <= j; ++i) col[i] = hh[i] + hh[kMaxM + 1 + i];
      const double w0 = std::sqrt(hh[2 * (kMaxM + 1)]), hn = std::sqrt(hh[2 * (kMaxM + 1) + 1]);
      col[j + 1] = hn;
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = t;
      }
      const double den = std::hypot(col[j], col[j + 1]);
      cs[j] = col[j] / den;
      sn[j] = col[j + 1] / den;
      col[j] = den;
      col[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      S.r_final = std::fabs(g[j + 1]);
      S.iters++;
      k = j + 1;
      if (!std::isfinite(S.r_final) || !std::isfinite(den) || den == 0.0) {
        bad = true;
        break;
      }
      if (S.r_final <= target || !(hn > 1e-14 * w0)) {  // converged, or an invariant Krylov space
        conv = true;
        break;
      }
      if (S.iters >= max_iters) break;
      FR3_TRY(lin(W.V + (size_t)(j + 1) * n, {{W.w, 1.0 / hn}}, n, s));
    }
    if (bad) {
      result = FR_ENAN;
      break;
    }
    // x += Z y with the triangular H y = g
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int l = i + 1; l < k; ++l) t -= H[(size_t)l * (m + 1) + i] * y[l];
      y[i] = t / H[(size_t)i * (m + 1) + i];
    }
    FR_HIP(hipMemcpyAsync(W.hd + 2 * (kMaxM + 1) + 2, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k3_maxpy, dim3(grid_of(n, 4096)), dim3(256), 0, s, x, W.Z, k, W.hd + 2 * (kMaxM + 1) + 2,
                       1.0, n);
    FR_HIP(hipGetLastError());
    FR_HIP(hipStreamSynchronize(s));  // y is read by the kernel before the host vector changes
    if (conv) {
      S.converged = 1;
      result = FR_OK;
      break;
    }
    FR3_TRY(jf(d, a, x, W.w, W, &evals, s));
    FR3_TRY(lin(W.r, {{b, 1.0}, {W.w, -1.0}}, n, s));
    FR3_TRY(norm(d, W.r, W, &beta, s));
    S.r_final = beta;
    if (!std::isfinite(beta)) {
      result = FR_ENAN;
    } else if (beta <= target) {
      S.converged = 1;
      result = FR_OK;
    } else if (S.iters >= max_iters) {
      result = FR_NOTCONV;
      break;
    } else {
      S.restarts++;
    }
  }
  S.residual_evals = evals;
  *out = S;
  return result;
}

// ---------------------------------------------------------------- PTC and the steps
// F(q) = (q - cst)/(omega dt) - R(q) = 0 by pseudo-transient continuation, in place on
// q; Rq holds R(q) on entry and exit.  The preconditioner is formed at every iterate.
fr_status ptc(const fr3d_disc* d, const double* cst, double omega_dt, double dt, double* q, double* Rq,
              const fr_solver_opts& o, W3& W, fr_step_stats* st, hipStream_t s) {
  const size_t n = d->ndof;
  double* negF = W.vec[9];
  double* dq = W.vec[10];
  const double iw = 1.0 / omega_dt;
  FR3_TRY(lin(negF, {{cst, iw}, {q, -iw}, {Rq, 1.0}}, n, s));
  double nF = 0.0;
  FR3_TRY(norm(d, negF, W, &nF, s));
  const double nF0 = nF;
  double dtau = o.dtau_init > 0 ? o.dtau_init : dt;
  double dtau_max = o.dtau_max > 0 ? o.dtau_max : 1e20;
  const int max_ptc = o.max_ptc > 0 ? o.max_ptc : 200;
  const int max_rej = o.max_reject > 0 ? o.max_reject : 30;
  int k = 0, rejects = 0;
  while (!(nF <= o.tol_nl * nF0)) {
    if (!std::isfinite(nF)) return FR_ENAN;
    if (k >= max_ptc) return FR_NOTCONV;
    if (rejects > max_rej) return FR_REJECTED;
    const double shift = 1.0 / dtau + iw;
    FR3_TRY(factor(d, q, Rq, shift, o.precond_precision, W, s));
    FR3_TRY(lin(dq, {}, n, s));
    fr_gmres_stats gs{};
    const JfArgs a{q, Rq, shift, o.lin.eps > 0 ? o.lin.eps : 1e-8, o.lin.eps_mode};
    fr_status g = gmres(d, W.inv, o.precond_precision, a, negF, dq, true, o.lin, &gs, W, s);
    if (g < 0) return g;
    st->gmres_iters += gs.iters;
    st->linear_solves++;
    st->residual_evals += gs.residual_evals + (long)colour_count(d) * 5 * d->np;
    if (!gs.converged) st->unconverged++;
    if (g == FR_ENAN) return FR_ENAN;
    if (!(gs.r_final <= 0.1 * gs.r_ref)) {  // GMRES did not gain one order of magnitude
      st->rejections++;
      rejects++;
      dtau_max *= 0.5;
      dtau = std::min(dtau, dtau_max);
      continue;
    }
    FR3_TRY(lin(q, {{q, 1.0}, {dq, 1.0}}, n, s));
    FR3_TRY(residual(d, q, Rq, W, s));
    st->residual_evals++;
    FR3_TRY(lin(negF, {{cst, iw}, {q, -iw}, {Rq, 1.0}}, n, s));
    double nFn = 0.0;
    FR3_TRY(norm(d, negF, W, &nFn, s));
    dtau = (nFn > 0.0) ? std::min(dtau * nF / nFn, dtau_max) : dtau_max;
    nF = nFn;
    ++k;
    st->ptc_iters++;
  }
  return FR_OK;
}

fr_status check_opts(const fr3d_disc* d, const fr_solver_opts& o) {
  if (d->p != 2 && d->p != 3) return set_error(FR_EINVAL, "3D implicit steps: p must be 2 or 3");
  if (o.lin.m < 1 || o.lin.m > kMaxM) return set_error(FR_EINVAL, "3D implicit steps: m must be 1 .. 64");
  if (o.lin.precond != FR_PC_EJACOBI || (o.precond_precision != FR_F64 && o.precond_precision != FR_F32))
    return set_error(FR_EINVAL, "3D implicit steps: element-Jacobi (FR_F64 or FR_F32) only");
  if (o.warm != nullptr || o.log != nullptr || o.d_yhist != nullptr)
    return set_error(FR_EINVAL, "3D implicit steps: no learned starts");
  if (o.lin.eps_mode != FR_EPS_RMS && o.lin.eps_mode != FR_EPS_ABS)
    return set_error(FR_EINVAL, "3D implicit steps: bad eps_mode");
  return FR_OK;
}

}  // namespace

size_t fr3d_step_bytes(const fr3d_disc* d, int m) { return carve_bytes(d, m); }
size_t fr3d_block_bytes(const fr3d_disc* d) { return block_store(d); }

fr_status fr3d_assemble_impl(const fr3d_disc* d, const double* U, double shift, double* blocks, void* work,
                             hipStream_t s) {
  if (d->p != 2 && d->p != 3) return set_error(FR_EINVAL, "3D element-Jacobi: p must be 2 or 3");
  W3 W = carve(d, work, 1);
  FR3_TRY(residual(d, U, W.vec[0], W, s));
  return assemble(d, U, W.vec[0], shift, blocks, FR_F64, W, s);
}

fr_status fr3d_factor_impl(const fr3d_disc* d, const double* U, double shift, double* inv, void* work,
                           hipStream_t s) {
  if (d->p != 2 && d->p != 3) return set_error(FR_EINVAL, "3D element-Jacobi: p must be 2 or 3");
  W3 W = carve(d, work, 1);
  FR3_TRY(residual(d, U, W.vec[0], W, s));
  FR3_TRY(assemble(d, U, W.vec[0], shift, W.blocks, FR_F64, W, s));
  return invert(d, W.blocks, inv, FR_F64, s);
}

fr_status fr3d_apply_impl(const fr3d_disc* d, const double* inv, const double* r, double* z, hipStream_t s) {
  return apply(d, inv, FR_F64, r, z, s);
}

fr_status fr3d_gmres_impl(const fr3d_disc* d, const double* inv, const double* U, const double* R0, double shift,
                          const double* b, double* x, const fr_gmres_opts& o, fr_gmres_stats* st, void* work,
                          hipStream_t s) {
  if (o.m < 1 || o.m > kMaxM) return set_error(FR_EINVAL, "fr3d_gmres_solve: m must be 1 .. 64");
  if (o.precond != FR_PC_EJACOBI) return set_error(FR_EINVAL, "fr3d_gmres_solve: element-Jacobi only");
  if (o.eps_mode != FR_EPS_RMS && o.eps_mode != FR_EPS_ABS) return set_error(FR_EINVAL, "fr3d_gmres_solve: bad eps_mode");
  W3 W = carve(d, work, o.m);
  const JfArgs a{U, R0, shift, o.eps > 0 ? o.eps : 1e-8, o.eps_mode};
  fr_status g = gmres(d, inv, FR_F64, a, b, x, false, o, st, W, s);
  FR_HIP(hipStreamSynchronize(s));
  return g;
}

fr_status fr3d_row_impl(const fr3d_disc* d, int scheme, double dt, double* U, const fr_solver_opts& o,
                        fr_step_stats* st, void* work, hipStream_t s) {
  FR3_TRY(check_opts(d, o));
  const RowScheme* T = row_scheme(scheme);
  if (T == nullptr) return set_error(FR_EINVAL, "fr3d_row_step: unknown scheme");
  const size_t n = d->ndof;
  const double t0 = now();
  W3 W = carve(d, work, o.lin.m);
  double* R0 = W.vec[0];
  double* Ui = W.vec[1];
  double* rhs = W.vec[2];
  double** Y = W.vec + 3;  // up to 6 stage increments: vec[3 .. 8]
  FR3_TRY(residual(d, U, R0, W, s));
  st->residual_evals++;
  const double shift = 1.0 / (T->gamma * dt);
  FR3_TRY(factor(d, U, R0, shift, o.precond_precision, W, s));
  st->residual_evals += (long)colour_count(d) * 5 * d->np;
  const JfArgs a{U, R0, shift, o.lin.eps > 0 ? o.lin.eps : 1e-8, o.lin.eps_mode};
  fr_status worst = FR_OK;
  for (int i = 0; i < T->s; ++i) {
    if (i == 0) {
      FR3_TRY(lin(rhs, {{R0, 1.0}}, n, s));
    } else {
      const double* xs[8];
      double cs[8];
      int k = 0;
      xs[k] = U;
      cs[k++] = 1.0;
      bool any = false;
      for (int j = 0; j < i; ++j)
        if (T->a[i][j] != 0.0) {
          xs[k] = Y[j];
          cs[k++] = T->a[i][j];
          any = true;
        }
      if (any) {
        FR_HIP(launch_lincomb(Ui, k, xs, cs, n, s));
        FR3_TRY(residual(d, Ui, rhs, W, s));
        st->residual_evals++;
      } else {
        FR3_TRY(lin(rhs, {{R0, 1.0}}, n, s));
      }
      k = 0;
      xs[k] = rhs;
      cs[k++] = 1.0;
      for (int j = 0; j < i; ++j)
        if (T->c[i][j] != 0.0) {
          xs[k] = Y[j];
          cs[k++] = T->c[i][j] / dt;
        }
      if (k > 1) FR_HIP(launch_lincomb(rhs, k, xs, cs, n, s));
    }
    FR3_TRY(lin(Y[i], {}, n, s));
    fr_gmres_stats gs{};
    fr_status g = gmres(d, W.inv, o.precond_precision, a, rhs, Y[i], true, o.lin, &gs, W, s);
    if (g < 0) return g;
    st->gmres_iters += gs.iters;
    st->linear_solves++;
    st->residual_evals += gs.residual_evals;
    if (g != FR_OK) {
      st->unconverged++;
      if (worst == FR_OK || g == FR_ENAN) worst = g;
    }
  }
  if (worst == FR_OK || (o.commit_unconverged && worst != FR_ENAN)) {
    const double* xs[8];
    double cs[8];
    int k = 0;
    xs[k] = U;
    cs[k++] = 1.0;
    for (int j = 0; j < T->s; ++j) {
      xs[k] = Y[j];
      cs[k++] = T->m[j];
    }
    FR_HIP(launch_lincomb(U, k, xs, cs, n, s));
  }
  FR_HIP(hipStreamSynchronize(s));
  st->wall_s = now() - t0;
  return worst;
}

fr_status fr3d_esdirk_impl(const fr3d_disc* d, int scheme, double dt, double* U, const fr_solver_opts& o,
                           fr_step_stats* st, void* work, hipStream_t s) {
  FR3_TRY(check_opts(d, o));
  const EsdirkScheme* T = esdirk_scheme(scheme);
  if (T == nullptr) return set_error(FR_EINVAL, "fr3d_esdirk_step: unknown scheme");
  if (T->s > 7) return set_error(FR_EINVAL, "fr3d_esdirk_step: too many stages");
  const size_t n = d->ndof;
  const double t0 = now();
  W3 W = carve(d, work, o.lin.m);
  double** Rj = W.vec;  // vec[0 .. 5]: R(q_j)
  double* q = W.vec[6];
  double* cst = W.vec[7];
  FR3_TRY(residual(d, U, Rj[0], W, s));
  st->residual_evals++;
  FR3_TRY(lin(q, {{U, 1.0}}, n, s));
  fr_status worst = FR_OK;
  for (int i = 1; i < T->s; ++i) {
    const double* xs[8];
    double cs[8];
    int k = 0;
    xs[k] = U;
    cs[k++] = 1.0;
    for (int j = 0; j < i; ++j)
      if (T->a[i][j] != 0.0) {
        xs[k] = Rj[j];
        cs[k++] = dt * T->a[i][j];
      }
    FR_HIP(launch_lincomb(cst, k, xs, cs, n, s));
    FR3_TRY(lin(Rj[i], {{Rj[i - 1], 1.0}}, n, s));  // R at the stage's start q_{i-1}
    fr_status p = ptc(d, cst, T->gamma * dt, dt, q, Rj[i], o, W, st, s);
    if (p < 0) return p;
    if (p != FR_OK && worst == FR_OK) worst = p;
    if (p == FR_ENAN || (p != FR_OK && !o.commit_unconverged)) break;
  }
  if (worst == FR_OK || (o.commit_unconverged && worst != FR_ENAN)) {
    const double* xs[8];
    double cs[8];
    int k = 0;
    xs[k] = U;
    cs[k++] = 1.0;
    for (int i = 0; i < T->s; ++i)
      if (T->b[i] != 0.0) {
        xs[k] = Rj[i];
        cs[k++] = dt * T->b[i];
      }
    FR_HIP(launch_lincomb(U, k, xs, cs, n, s));
  }
  FR_HIP(hipStreamSynchronize(s));
  st->wall_s = now() - t0;
  return worst;
}

fr_status fr3d_bdf2_impl(const fr3d_disc* d, double dt, const double* Unm1, const double* Un, double* Unp1,
                         const fr_solver_opts& o, fr_step_stats* st, void* work, hipStream_t s) {
  FR3_TRY(check_opts(d, o));
  const size_t n = d->ndof;
  const double t0 = now();
  W3 W = carve(d, work, o.lin.m);
  double* q = W.vec[0];
  double* Rq = W.vec[1];
  double* cst = W.vec[2];
  double omega;
  if (Unm1 == nullptr) {
    omega = 1.0;
    FR3_TRY(lin(cst, {{Un, 1.0}}, n, s));
  } else {
    omega = 2.0 / 3.0;
    FR3_TRY(lin(cst, {{Un, 4.0 / 3.0}, {Unm1, -1.0 / 3.0}}, n, s));
  }
  FR3_TRY(lin(q, {{Un, 1.0}}, n, s));
  FR3_TRY(residual(d, q, Rq, W, s));
  st->residual_evals++;
  fr_status p = ptc(d, cst, omega * dt, dt, q, Rq, o, W, st, s);
  if (p < 0) return p;
  if (p == FR_OK || (o.commit_unconverged && p != FR_ENAN)) FR3_TRY(lin(Unp1, {{q, 1.0}}, n, s));
  FR_HIP(hipStreamSynchronize(s));
  st->wall_s = now() - t0;
  return p;
}

}  // namespace frjf
