// FR/CPR residual of the 2D Euler equations (Section 3) and the fused
// Jacobian-free product (Section 4.5), one kernel template:
//   MODE 0: out = R(U)
//   MODE 1: out = shift v - [R(U + e v) - R0] / e
//   MODE 2: out = b - (shift v - [R(U + e v) - R0] / e)      (GMRES true residual)
//
// A workgroup owns a TX x TY tile of elements.  Phase 1 evaluates the
// transformed fluxes F = y_eta f - x_eta g, G = -y_xi f + x_xi g at every
// solution point into LDS.  Phase 2 forms, for every face point of every
// element, the element's own solution/flux traces, the neighbour's solution
// trace (from LDS inside the tile, from global memory for the halo), and the
// common flux |S| f^com with the state on the -xi / -eta side first; each
// element recomputes its four faces with identical arguments to its
// neighbours, so both sides of a face see the same numerical flux and the
// scheme stays conservative without atomics.  Phase 3 applies the derivative
// matrix and the Radau correction derivatives.
#include "internal.h"
#include "physics.h"

namespace frjf {

#ifndef FRJF_TILE_P2
#define FRJF_TILE_P2 8, 4, 320
#endif
#ifndef FRJF_TILE_P3
#define FRJF_TILE_P3 4, 4, 256
#endif
#ifndef FRJF_TILE_P4
#define FRJF_TILE_P4 5, 2, 256
#endif

template <int TX_, int TY_, int NT_>
struct TileShape {
  static constexpr int TX = TX_, TY = TY_, NT = NT_;
};
template <int P>
struct EulerTile;
template <>
struct EulerTile<2> : TileShape<FRJF_TILE_P2> {};
template <>
struct EulerTile<3> : TileShape<FRJF_TILE_P3> {};
template <>
struct EulerTile<4> : TileShape<FRJF_TILE_P4> {};

// Tiles handed to the 8 XCDs in contiguous ranges (workgroup i runs on XCD i % 8),
// so neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_remap(int i, int T) {
  const int q = T >> 3, r = T & 7;
  const int x = i & 7, l = i >> 3;
  return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

struct MeshArgs {
  const double* nodes;
  int nx, ny, nel;
  double gam;
};

template <int MODE>
__device__ __forceinline__ double state_at(const ResArgs& a, size_t gi, double e) {
  if constexpr (MODE == 0)
    return a.U[gi];
  else
    return fma(e, a.V[gi], a.U[gi]);
}

template <int FLUX>
__device__ __forceinline__ void face_common_flux(const double qL[4], const double qR[4], double Sx, double Sy,
                                                 double gam, double out[4]) {
  if constexpr (FLUX == 0)
    rusanov_flux_S(qL, qR, Sx, Sy, sqrt(Sx * Sx + Sy * Sy), gam, out);
  else
    roe_flux(qL, qR, Sx, Sy, gam, out);
}

template <int P, int FLUX, int MODE>
__global__ void __launch_bounds__(EulerTile<P>::NT) k_euler(const ResArgs a, const MeshArgs g, const Basis B) {
  constexpr int n = P + 1, Np = n * n;
  constexpr int TX = EulerTile<P>::TX, TY = EulerTile<P>::TY, NE = TX * TY, NT = EulerTile<P>::NT;
  constexpr int NFV = (TX + 1) * TY, NFH = TX * (TY + 1);  // xi-faces and eta-faces of the tile
  __shared__ double sQ[4][NE * Np];
  __shared__ double sF[4][NE * Np];
  __shared__ double sG[4][NE * Np];
  __shared__ double sIJ[NE * Np];
  __shared__ double sFv[4][NFV * n], sFh[4][NFH * n];   // common fluxes |S| f^com on the tile's faces
  __shared__ double sJmp[4][4][NE * n];                  // F^num - F^l on each element face
  __shared__ double sX[n], sD[n * n], sLm[n], sLp[n], sGL[n], sGR[n];

  if (MODE != 0 && a.skip != nullptr && *a.skip) return;
  const int tid = threadIdx.x;
  if (tid < n * n) sD[tid] = B.D[tid / n][tid % n];
  if (tid < n) {
    sX[tid] = B.x[tid];
    sLm[tid] = B.lm[tid];
    sLp[tid] = B.lp[tid];
    sGL[tid] = B.gL[tid];
    sGR[tid] = B.gR[tid];
  }
  const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + TY - 1) / TY;
  const int tile = xcd_remap(blockIdx.x, ntx * nty);
  const int ex0 = (tile % ntx) * TX, ey0 = (tile / ntx) * TY;
  const size_t nel = (size_t)g.nel;
  double e = 0.0;
  bool zero_v = false;
  if constexpr (MODE != 0) {
    if (a.eps_mode == FR_EPS_RMS) {
      const double n2 = *a.nrm2;
      if (n2 > 0.0)
        e = a.eps / sqrt(n2 / (double)(4 * nel * Np));
      else
        zero_v = true;
    } else {
      e = a.eps;
    }
  }
  __syncthreads();

  // ---- phase 1: transformed fluxes at the solution points
  for (int idx = tid; idx < NE * Np; idx += NT) {
    const int le = idx / Np, k = idx - le * Np;
    const int ex = ex0 + le % TX, ey = ey0 + le / TX;
    if (ex >= g.nx || ey >= g.ny) continue;
    const size_t el = (size_t)ey * g.nx + ex;
    double q[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) q[v] = state_at<MODE>(a, ((size_t)v * nel + el) * Np + k, e);
    double c[8];
    load_corners(g.nodes, g.nx, ex, ey, c);
    const Metric m = bilinear_metric(c, sX[k % n], sX[k / n]);
    double f[4], gg[4];
    euler_fluxes(q, g.gam, f, gg);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sQ[v][idx] = q[v];
      sF[v][idx] = m.yeta * f[v] - m.xeta * gg[v];
      sG[v][idx] = -m.yxi * f[v] + m.xxi * gg[v];
    }
    sIJ[idx] = 1.0 / m.J;
  }
  __syncthreads();

  // ---- phase 2a: one common flux per face point of the tile (the -xi / -eta side first)
  for (int idx = tid; idx < (NFV + NFH) * n; idx += NT) {
    const bool vert = idx < NFV * n;
    const int f = vert ? idx / n : (idx - NFV * n) / n;
    const int j = idx % n;
    int fx, fy, exA, eyA, exB, eyB;  // A: -side element, B: +side element (tile coordinates)
    if (vert) {
      fx = f % (TX + 1);
      fy = f / (TX + 1);
      exA = fx - 1;
      eyA = fy;
      exB = fx;
      eyB = fy;
    } else {
      fx = f % TX;
      fy = f / TX;
      exA = fx;
      eyA = fy - 1;
      exB = fx;
      eyB = fy;
    }
    // the face is needed if one of its elements belongs to the tile and the mesh
    const bool okA = exA >= 0 && exA < TX && eyA >= 0 && eyA < TY && ex0 + exA < g.nx && ey0 + eyA < g.ny;
    const bool okB = exB < TX && eyB < TY && ex0 + exB < g.nx && ey0 + eyB < g.ny;
    if (!okA && !okB) continue;
    double qs[2][4];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      int gx = ex0 + (side ? exB : exA), gy = ey0 + (side ? eyB : eyA);
      gx = (gx < 0) ? gx + g.nx : (gx >= g.nx ? gx - g.nx : gx);
      gy = (gy < 0) ? gy + g.ny : (gy >= g.ny ? gy - g.ny : gy);
      const double* lw = side ? sLm : sLp;  // the -side element's +face, the +side element's -face
      double qv[4] = {0, 0, 0, 0};
      if (gx >= ex0 && gx < ex0 + TX && gy >= ey0 && gy < ey0 + TY) {
        const int le = (gy - ey0) * TX + (gx - ex0);
#pragma unroll
        for (int c = 0; c < n; ++c) {
          const int kk = le * Np + (vert ? j * n + c : c * n + j);
#pragma unroll
          for (int v = 0; v < 4; ++v) qv[v] = fma(lw[c], sQ[v][kk], qv[v]);
        }
      } else {
        const size_t el = (size_t)gy * g.nx + gx;
#pragma unroll
        for (int c = 0; c < n; ++c) {
          const int kk = vert ? j * n + c : c * n + j;
#pragma unroll
          for (int v = 0; v < 4; ++v)
            qv[v] = fma(lw[c], state_at<MODE>(a, ((size_t)v * nel + el) * Np + kk, e), qv[v]);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) qs[side][v] = qv[v];
    }
    double Sx, Sy;
    if (vert) {
      const int ix = ex0 + fx;
      xi_face_normal(g.nodes, g.nx, ix >= g.nx ? ix - g.nx : ix, ey0 + fy, &Sx, &Sy);
    } else {
      const int iy = ey0 + fy;
      eta_face_normal(g.nodes, g.nx, ex0 + fx, iy >= g.ny ? iy - g.ny : iy, &Sx, &Sy);
    }
    double Fn[4];
    face_common_flux<FLUX>(qs[0], qs[1], Sx, Sy, g.gam, Fn);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (vert)
        sFv[v][f * n + j] = Fn[v];
      else
        sFh[v][f * n + j] = Fn[v];
    }
  }
  __syncthreads();

  // ---- phase 2b: jumps F^num - F^l on the four faces of every element
  for (int idx = tid; idx < NE * 4 * n; idx += NT) {
    const int le = idx / (4 * n);
    const int r = idx - le * 4 * n;
    const int fc = r / n, j = r - fc * n;
    const int lx = le % TX, ly = le / TX;
    if (ex0 + lx >= g.nx || ey0 + ly >= g.ny) continue;
    const bool xi_face = fc < 2;
    const double* lw = (fc == 0 || fc == 2) ? sLm : sLp;
    double Fl[4] = {0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < n; ++c) {
      const int kk = le * Np + (xi_face ? j * n + c : c * n + j);
#pragma unroll
      for (int v = 0; v < 4; ++v) Fl[v] = fma(lw[c], xi_face ? sF[v][kk] : sG[v][kk], Fl[v]);
    }
    int fi;
    if (fc == 0) fi = ly * (TX + 1) + lx;
    else if (fc == 1) fi = ly * (TX + 1) + lx + 1;
    else if (fc == 2) fi = ly * TX + lx;
    else fi = (ly + 1) * TX + lx;
#pragma unroll
    for (int v = 0; v < 4; ++v) sJmp[fc][v][le * n + j] = (xi_face ? sFv[v][fi * n + j] : sFh[v][fi * n + j]) - Fl[v];
  }
  __syncthreads();

  // ---- phase 3: divergence of the corrected flux
  for (int idx = tid; idx < NE * Np; idx += NT) {
    const int le = idx / Np, k = idx - le * Np;
    const int ex = ex0 + le % TX, ey = ey0 + le / TX;
    if (ex >= g.nx || ey >= g.ny) continue;
    const int ia = k % n, ib = k / n;
    const size_t el = (size_t)ey * g.nx + ex;
    const int rowb = le * Np + ib * n, cola = le * Np + ia;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double div = 0.0;
#pragma unroll
      for (int c = 0; c < n; ++c) {
        div = fma(sD[ia * n + c], sF[v][rowb + c], div);
        div = fma(sD[ib * n + c], sG[v][cola + c * n], div);
      }
      div = fma(sJmp[0][v][le * n + ib], sGL[ia], div);
      div = fma(sJmp[1][v][le * n + ib], sGR[ia], div);
      div = fma(sJmp[2][v][le * n + ia], sGL[ib], div);
      div = fma(sJmp[3][v][le * n + ia], sGR[ib], div);
      const double R = -div * sIJ[idx];
      const size_t gi = ((size_t)v * nel + el) * Np + k;
      if constexpr (MODE == 0) {
        a.out[gi] = R;
      } else {
        const double av = zero_v ? 0.0 : a.shift * a.V[gi] - (R - a.R0[gi]) / e;
        if constexpr (MODE == 1)
          a.out[gi] = av;
        else
          a.out[gi] = a.B[gi] - av;
      }
    }
  }
}

template <int P, int FLUX>
static hipError_t launch_euler_pf(const fr_disc* d, int mode, const ResArgs& a, hipStream_t s) {
  using T = EulerTile<P>;
  const int ntx = (d->nx + T::TX - 1) / T::TX, nty = (d->ny + T::TY - 1) / T::TY;
  const MeshArgs g{d->nodes, d->nx, d->ny, d->nel, d->phys.gamma};
  dim3 grid(ntx * nty), block(T::NT);
  if (mode == 0)
    hipLaunchKernelGGL((k_euler<P, FLUX, 0>), grid, block, 0, s, a, g, d->basis);
  else if (mode == 1)
    hipLaunchKernelGGL((k_euler<P, FLUX, 1>), grid, block, 0, s, a, g, d->basis);
  else
    hipLaunchKernelGGL((k_euler<P, FLUX, 2>), grid, block, 0, s, a, g, d->basis);
  return hipGetLastError();
}

template <int P>
static hipError_t launch_euler_p(const fr_disc* d, int mode, const ResArgs& a, hipStream_t s) {
  return d->flux == FR_ROE ? launch_euler_pf<P, 1>(d, mode, a, s) : launch_euler_pf<P, 0>(d, mode, a, s);
}

hipError_t launch_ns_residual(const fr_disc* d, int mode, const ResArgs& a, hipStream_t s);

hipError_t launch_residual(const fr_disc* d, int mode, const ResArgs& a, hipStream_t s) {
  if (d->physics == FR_NS_BR1) return launch_ns_residual(d, mode, a, s);
  switch (d->p) {
    case 2: return launch_euler_p<2>(d, mode, a, s);
    case 3: return launch_euler_p<3>(d, mode, a, s);
    case 4: return launch_euler_p<4>(d, mode, a, s);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- solution points
__global__ void k_solution_points(const MeshArgs g, const Basis B, double* xy) {
  const int n = B.n, Np = n * n;
  const size_t total = (size_t)g.nel * Np;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int el = (int)(i / Np), k = (int)(i % Np);
    const int ex = el % g.nx, ey = el / g.nx;
    double c[8];
    load_corners(g.nodes, g.nx, ex, ey, c);
    const double xi = B.x[k % n], eta = B.x[k / n];
    const double w00 = 0.25 * (1 - xi) * (1 - eta), w10 = 0.25 * (1 + xi) * (1 - eta);
    const double w01 = 0.25 * (1 - xi) * (1 + eta), w11 = 0.25 * (1 + xi) * (1 + eta);
    xy[i] = w00 * c[0] + w10 * c[2] + w01 * c[4] + w11 * c[6];
    xy[total + i] = w00 * c[1] + w10 * c[3] + w01 * c[5] + w11 * c[7];
  }
}

hipError_t launch_solution_points(const fr_disc* d, double* xy, hipStream_t s) {
  const MeshArgs g{d->nodes, d->nx, d->ny, d->nel, d->phys.gamma};
  hipLaunchKernelGGL(k_solution_points, dim3(512), dim3(256), 0, s, g, d->basis, xy);
  return hipGetLastError();
}

}  // namespace frjf

namespace frjf {

// ---------------------------------------------------------------- L2 error against the exact vortex
// Section 5.1: sqrt( int (s_exact - s_num)^2 dV / V ), Gauss quadrature at the solution points.
// prm: rho_inf, u_inf, v_inf, p_inf, R, gamma, alpha, phi, xc, yc, xlo, ylo, Lx, Ly.
struct VortexPrm {
  double v[14];
};

__device__ double wrap_periodic(double d, double L) { return d - L * floor(d / L + 0.5); }

__global__ void __launch_bounds__(256) k_l2_vortex(const MeshArgs g, const Basis B, const double* __restrict__ U,
                                                   int var, double t, VortexPrm P, double* partials) {
  const int n = B.n, Np = n * n;
  const size_t total = (size_t)g.nel * Np;
  double acc[2] = {0.0, 0.0};
  const double* p = P.v;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int el = (int)(i / Np), k = (int)(i % Np);
    const int ex = el % g.nx, ey = el / g.nx;
    double c[8];
    load_corners(g.nodes, g.nx, ex, ey, c);
    const double xi = B.x[k % n], eta = B.x[k / n];
    const Metric m = bilinear_metric(c, xi, eta);
    const double w00 = 0.25 * (1 - xi) * (1 - eta), w10 = 0.25 * (1 + xi) * (1 - eta);
    const double w01 = 0.25 * (1 - xi) * (1 + eta), w11 = 0.25 * (1 + xi) * (1 + eta);
    const double x = w00 * c[0] + w10 * c[2] + w01 * c[4] + w11 * c[6];
    const double y = w00 * c[1] + w10 * c[3] + w01 * c[5] + w11 * c[7];
    const double xb = wrap_periodic(x - p[8] - p[1] * t, p[12]);
    const double yb = wrap_periodic(y - p[9] - p[2] * t, p[13]);
    const double r2 = xb * xb + yb * yb;
    const double ex_ = exp(p[7] * (1.0 - r2));
    const double tinf = p[3] / (p[0] * p[4]);
    const double dT = -(p[6] * p[6]) * (p[5] - 1.0) / (16.0 * p[7] * p[5] * M_PI * M_PI) * ex_ * ex_;
    const double rho = p[0] * pow((tinf + dT) / tinf, 1.0 / (p[5] - 1.0));
    double s_ex, s_num;
    const size_t el_ = (size_t)el;
    const double rnum = U[el_ * Np + k];
    if (var == 0) {
      s_ex = rho;
      s_num = rnum;
    } else {
      s_ex = p[1] - p[6] / (2.0 * M_PI) * yb * ex_;
      s_num = U[((size_t)g.nel + el_) * Np + k] / rnum;
    }
    const double wq = B.w[k % n] * B.w[k / n] * m.J;
    const double dd = s_ex - s_num;
    acc[0] = fma(wq * dd, dd, acc[0]);
    acc[1] += wq;
  }
  __shared__ double red[4][2];
  for (int q = 0; q < 2; ++q) {
    double t = acc[q];
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = t;
  }
  __syncthreads();
  if (threadIdx.x < 2)
    partials[blockIdx.x * 2 + threadIdx.x] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

hipError_t launch_l2_vortex(const fr_disc* d, const double* U, int var, double t, const double* prm,
                            double* partials, unsigned* counter, double* out, hipStream_t s) {
  const MeshArgs g{d->nodes, d->nx, d->ny, d->nel, d->phys.gamma};
  VortexPrm P;
  for (int i = 0; i < 14; ++i) P.v[i] = prm[i];
  hipLaunchKernelGGL(k_l2_vortex, dim3(256), dim3(256), 0, s, g, d->basis, U, var, t, P, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(partials, 256, 2, 2, out, nullptr, s);
}

}  // namespace frjf
