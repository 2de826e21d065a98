// FR on hexahedra for the 3D compressible Navier-Stokes equations (Euler when mu = 0),
// Section 3's hexahedral forms on uniform Cartesian elements of a triply periodic box
// (the Taylor-Green vortex of Section 5.3), with the BR2 common gradient (Section 3,
// eq. com_grad_q and its lifting with the (P+1)(P+2)/2 penalty).
//
// Layout: U[v][e][k], v = 0..4 (rho, rho u, rho v, rho w, E), e = (ez ny + ey) nx + ex,
// k = (c n + b) n + a with a along x, b along y, c along z.  Face f = 2 d + s of axis d,
// s = 0 at -1 and 1 at +1; the n^2 points of a face are j = (second remaining axis) n +
// (first remaining axis): d = 0 -> j = c n + b, d = 1 -> j = c n + a, d = 2 -> j = b n + a.
// The map is affine: d/dx_d = (2/h_d) d/dxi_d, and the residual is
//   R = -sum_d (2/h_d) [ D f_d + (f^com - f^l)_{s=0} g_L' + (f^com - f^l)_{s=1} g_R' ]
// with f_d the inviscid minus viscous flux along axis d.
//
// Kernel A (k3_faces): per element, its solution traces on the six faces and, with
//   viscosity, the raw gradient of its solution polynomial (no corrections) extrapolated
//   there: T[e][f][v][j], G[e][f][v][j][x|y|z].
// Kernel B (k3_res): per element, the common states (q_own + q_nbr)/2 from T, the
//   FR-corrected gradient at the solution points, the total fluxes there, the common
//   fluxes on the faces (Riemann solver between the traces; viscous flux at the common
//   state with the BR2 common gradient: the mean of each side's G plus its lifting
//   r = c_P (q^com - q_side) (2/h_d) n_out), and R.
// MODE 0: out = R(U); MODE 1: out = shift v - (R(U + e v) - R0) / e (Jacobian-free product).
#include <cmath>
#include <vector>

#include "internal.h"
#include "wavesum.h"

namespace frjf {

struct Args3 {
  const double* U;
  const double* V;
  const double* R0;
  double* out;
  double* T;  // traces [nel][6][5][n^2]
  double* G;  // raw face gradients [nel][6][5][n^2][3]
  const double* nrm2;
  const int* elist;  // null: workgroup b is element b; else element elist[b]
  size_t cs;         // copies (blockIdx.y): state and output stride in doubles,
  size_t fs;         // and face-data stride in bytes (0 with one copy)
  double eps, shift;
  int eps_mode;
  int nx, ny, nz, nel;
  double h[3];
  double gamma, rgas, mu, cp_over_pr;
};

template <int P>
struct C3 {
  static constexpr int n = P + 1, n2 = n * n, Np = n * n * n, NF = 6 * n2;
  static constexpr int NT = (P <= 3) ? 64 : 128;
};

// ---------------------------------------------------------------- 3D physics
__device__ __forceinline__ double p3(const double q[5], double gam) {
  return (gam - 1.0) * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
}

// inviscid flux along axis d
__device__ __forceinline__ void inv3(const double q[5], int d, double gam, double f[5]) {
  const double vel = q[1 + d] / q[0];
  const double p = p3(q, gam);
  f[0] = q[1 + d];
  f[1] = q[1] * vel;
  f[2] = q[2] * vel;
  f[3] = q[3] * vel;
  f[4] = vel * (q[4] + p);
  f[1 + d] += p;
}

// viscous flux along axis d from q and its gradient g[k][v] = dq_v/dx_k (zero bulk viscosity)
__device__ __forceinline__ void vis3(const double q[5], const double g[3][5], int d, const Args3& a, double f[5]) {
  const double ir = 1.0 / q[0];
  const double u[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
  double du[3][3];  // du[i][k] = du_i / dx_k
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) du[i][k] = (g[k][1 + i] - u[i] * g[k][0]) * ir;
  const double ke = 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const double p = (a.gamma - 1.0) * (q[4] - q[0] * ke);
  const double T = p * ir / a.rgas;
  const double dpd = (a.gamma - 1.0) * (g[d][4] - ke * g[d][0] - q[0] * (u[0] * du[0][d] + u[1] * du[1][d] + u[2] * du[2][d]));
  const double dTd = (dpd - a.rgas * T * g[d][0]) * ir / a.rgas;
  const double div = du[0][0] + du[1][1] + du[2][2];
  double tau[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) tau[i] = a.mu * (du[i][d] + du[d][i] - ((i == d) ? (2.0 / 3.0) * div : 0.0));
  f[0] = 0.0;
  f[1] = tau[0];
  f[2] = tau[1];
  f[3] = tau[2];
  f[4] = u[0] * tau[0] + u[1] * tau[1] + u[2] * tau[2] + a.mu * a.cp_over_pr * dTd;
}

// common inviscid flux along +axis d between the left (qL) and right (qR) traces
template <int FLUX>
__device__ __forceinline__ void riemann3(const double qL[5], const double qR[5], int d, double gam, double F[5]) {
  double fL[5], fR[5];
  inv3(qL, d, gam, fL);
  inv3(qR, d, gam, fR);
  if constexpr (FLUX == 0) {  // Rusanov: lambda = max(|u_d| + c) of the two sides
    const double sl = fabs(qL[1 + d] / qL[0]) + sqrt(gam * p3(qL, gam) / qL[0]);
    const double sr = fabs(qR[1 + d] / qR[0]) + sqrt(gam * p3(qR, gam) / qR[0]);
    const double lam = fmax(sl, sr);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * lam * (qR[v] - qL[v]);
  } else {  // Roe: acoustic, entropy and two shear waves at the Roe average, no entropy fix
    const double rL = qL[0], rR = qR[0];
    const double pL = p3(qL, gam), pR = p3(qR, gam);
    const double sL = sqrt(rL), sR = sqrt(rR), is = 1.0 / (sL + sR);
    double uL[3], uR[3], u[3], du[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      uL[i] = qL[1 + i] / rL;
      uR[i] = qR[1 + i] / rR;
      u[i] = (sL * uL[i] + sR * uR[i]) * is;
      du[i] = uR[i] - uL[i];
    }
    const double H = (sL * (qL[4] + pL) / rL + sR * (qR[4] + pR) / rR) * is;
    const double q2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double c = sqrt((gam - 1.0) * (H - 0.5 * q2));
    const double rho = sL * sR, un = u[d];
    const double dr = rR - rL, dp = pR - pL;
    const double a1 = (dp - rho * c * du[d]) / (2.0 * c * c);
    const double a2 = dr - dp / (c * c);
    const double a4 = (dp + rho * c * du[d]) / (2.0 * c * c);
    const double l1 = fabs(un - c), l2 = fabs(un), l4 = fabs(un + c);
    double diss[5];
    diss[0] = l1 * a1 + l2 * a2 + l4 * a4;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double e = (i == d) ? c : 0.0;
      diss[1 + i] = l1 * a1 * (u[i] - e) + l2 * a2 * u[i] + l4 * a4 * (u[i] + e);
    }
    diss[4] = l1 * a1 * (H - un * c) + l2 * a2 * 0.5 * q2 + l4 * a4 * (H + un * c);
#pragma unroll
    for (int t = 0; t < 3; ++t) {  // shear waves
      if (t == d) continue;
      const double st = l2 * rho * du[t];
      diss[1 + t] += st;
      diss[4] += st * u[t];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * diss[v];
  }
}

// ---------------------------------------------------------------- index helpers
// point of line (d; j) at position t along axis d
template <int n>
__device__ __forceinline__ int line_pt(int d, int j, int t) {
  const int i0 = j % n, i1 = j / n;
  return d == 0 ? (i1 * n + i0) * n + t : (d == 1 ? (i1 * n + t) * n + i0 : (t * n + i1) * n + i0);
}
// face point j on axis-d faces through point k, and k's position along d
template <int n>
__device__ __forceinline__ void point_on_line(int k, int d, int* j, int* t) {
  const int a = k % n, b = (k / n) % n, c = k / (n * n);
  if (d == 0) {
    *j = c * n + b;
    *t = a;
  } else if (d == 1) {
    *j = c * n + a;
    *t = b;
  } else {
    *j = b * n + a;
    *t = c;
  }
}
__device__ __forceinline__ int nbr3(const Args3& a, int e, int d, int s) {
  int ex = e % a.nx, ey = (e / a.nx) % a.ny, ez = e / (a.nx * a.ny);
  const int step = s ? 1 : -1;
  if (d == 0) ex = (ex + step + a.nx) % a.nx;
  if (d == 1) ey = (ey + step + a.ny) % a.ny;
  if (d == 2) ez = (ez + step + a.nz) % a.nz;
  return (ez * a.ny + ey) * a.nx + ex;
}
__device__ __forceinline__ size_t t_index(int e, int f, int v, int j, int n2) {
  return (((size_t)e * 6 + f) * 5 + v) * n2 + j;
}

template <int MODE>
__device__ __forceinline__ double state3(const double* U, const double* V, size_t gi, double e) {
  if constexpr (MODE == 0)
    return U[gi];
  else
    return fma(e, V[gi], U[gi]);
}

__device__ __forceinline__ double eps3(const Args3& a, size_t ndof, bool* zero_v) {
  *zero_v = false;
  if (a.eps_mode == FR_EPS_RMS) {
    const double n2 = *a.nrm2;
    if (n2 > 0.0) return a.eps / sqrt(n2 / (double)ndof);
    *zero_v = true;
    return 0.0;
  }
  return a.eps;
}

// ---------------------------------------------------------------- kernel A: traces and raw face gradients
template <int P, int MODE, bool VISC>
__global__ void __launch_bounds__(C3<P>::NT) k3_faces(const Args3 a, const Basis B) {
  // copy blockIdx.y (one copy unless a.cs, a.fs are set): its state and face data
  const size_t cy = blockIdx.y;
  const double* const Uc = a.U + cy * a.cs;
  double* const Tc = (double*)((char*)a.T + cy * a.fs);
  double* const Gc = a.G != nullptr ? (double*)((char*)a.G + cy * a.fs) : nullptr;
  using C = C3<P>;
  constexpr int n = C::n, n2 = C::n2, Np = C::Np, NF = C::NF, NT = C::NT;
  __shared__ double q[5][Np];
  __shared__ double gr[VISC ? 3 : 1][5][VISC ? Np : 1];
  const int el = a.elist != nullptr ? a.elist[blockIdx.x] : (int)blockIdx.x, tid = threadIdx.x;
  const size_t nel = (size_t)a.nel, ndof = 5 * nel * Np;
  bool zv = false;
  const double e = MODE ? eps3(a, ndof, &zv) : 0.0;
  for (int k = tid; k < Np; k += NT)
#pragma unroll
    for (int v = 0; v < 5; ++v) q[v][k] = state3<MODE>(Uc, a.V, ((size_t)v * nel + el) * Np + k, e);
  __syncthreads();
  if constexpr (VISC) {
    for (int k = tid; k < Np; k += NT) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        int j, t;
        point_on_line<n>(k, d, &j, &t);
        const double s = 2.0 / a.h[d];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          double x = 0.0;
          for (int m = 0; m < n; ++m) x = fma(B.D[t][m], q[v][line_pt<n>(d, j, m)], x);
          gr[d][v][k] = s * x;
        }
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < NF; idx += NT) {
    const int f = idx / n2, j = idx % n2, d = f >> 1;
    const double* lw = (f & 1) ? B.lp : B.lm;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double x = 0.0;
      for (int m = 0; m < n; ++m) x = fma(lw[m], q[v][line_pt<n>(d, j, m)], x);
      Tc[t_index(el, f, v, j, n2)] = x;
      if constexpr (VISC) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double y = 0.0;
          for (int m = 0; m < n; ++m) y = fma(lw[m], gr[c][v][line_pt<n>(d, j, m)], y);
          Gc[t_index(el, f, v, j, n2) * 3 + c] = y;
        }
      }
    }
  }
}

// ---------------------------------------------------------------- kernel B: residual
template <int P, int FLUX, int MODE, bool VISC>
__global__ void __launch_bounds__(C3<P>::NT) k3_res(const Args3 a, const Basis B) {
  // copy blockIdx.y (one copy unless a.cs, a.fs are set): its state, face data and output
  const size_t cy = blockIdx.y;
  const double* const Uc = a.U + cy * a.cs;
  const double* const Tc = (const double*)((const char*)a.T + cy * a.fs);
  const double* const Gc = a.G != nullptr ? (const double*)((const char*)a.G + cy * a.fs) : nullptr;
  double* const outc = a.out + cy * a.cs;
  using C = C3<P>;
  constexpr int n = C::n, n2 = C::n2, Np = C::Np, NF = C::NF, NT = C::NT;
  constexpr double cP = 0.5 * (P + 1) * (P + 2);
  __shared__ double q[5][Np];
  __shared__ double tr[6][5][n2];   // own traces, then the face jumps f^com - f^l
  __shared__ double tn[6][5][n2];   // neighbours' traces on the shared faces
  __shared__ double qc[6][5][n2];   // common states
  __shared__ double F[3][5][Np];    // corrected gradient, then the total fluxes
  const int el = a.elist != nullptr ? a.elist[blockIdx.x] : (int)blockIdx.x, tid = threadIdx.x;
  const size_t nel = (size_t)a.nel, ndof = 5 * nel * Np;
  bool zero_v = false;
  const double e = MODE ? eps3(a, ndof, &zero_v) : 0.0;
  for (int k = tid; k < Np; k += NT)
#pragma unroll
    for (int v = 0; v < 5; ++v) q[v][k] = state3<MODE>(Uc, a.V, ((size_t)v * nel + el) * Np + k, e);
  for (int idx = tid; idx < NF; idx += NT) {
    const int f = idx / n2, j = idx % n2, d = f >> 1, s = f & 1;
    const int ne = nbr3(a, el, d, s);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double o = Tc[t_index(el, f, v, j, n2)];
      const double m = Tc[t_index(ne, f ^ 1, v, j, n2)];
      tr[f][v][j] = o;
      tn[f][v][j] = m;
      qc[f][v][j] = 0.5 * (o + m);
    }
  }
  __syncthreads();
  // corrected gradient (viscous), then the total fluxes at the solution points
  for (int k = tid; k < Np; k += NT) {
    double qk[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) qk[v] = q[v][k];
    double g[3][5];
    if constexpr (VISC) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        int j, t;
        point_on_line<n>(k, d, &j, &t);
        const double s = 2.0 / a.h[d];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          double x = 0.0;
          for (int m = 0; m < n; ++m) x = fma(B.D[t][m], q[v][line_pt<n>(d, j, m)], x);
          x = fma(qc[2 * d][v][j] - tr[2 * d][v][j], B.gL[t], x);
          x = fma(qc[2 * d + 1][v][j] - tr[2 * d + 1][v][j], B.gR[t], x);
          g[d][v] = s * x;
        }
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double fi[5];
      inv3(qk, d, a.gamma, fi);
      if constexpr (VISC) {
        double fv[5];
        vis3(qk, g, d, a, fv);
#pragma unroll
        for (int v = 0; v < 5; ++v) fi[v] -= fv[v];
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) F[d][v][k] = fi[v];
    }
  }
  __syncthreads();
  // common fluxes and jumps on the faces
  for (int idx = tid; idx < NF; idx += NT) {
    const int f = idx / n2, j = idx % n2, d = f >> 1, s = f & 1;
    const double* lw = s ? B.lp : B.lm;
    double qo[5], qn[5], fc[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      qo[v] = tr[f][v][j];
      qn[v] = tn[f][v][j];
    }
    if (s == 0)
      riemann3<FLUX>(qn, qo, d, a.gamma, fc);
    else
      riemann3<FLUX>(qo, qn, d, a.gamma, fc);
    if constexpr (VISC) {
      const int ne = nbr3(a, el, d, s);
      double gc[3][5], qcv[5];
      const double sg = s ? 1.0 : -1.0;  // own outward normal along axis d; the neighbour's is opposite
      const double lift = cP * 2.0 / a.h[d];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        qcv[v] = qc[f][v][j];
        const size_t io = t_index(el, f, v, j, n2) * 3, in = t_index(ne, f ^ 1, v, j, n2) * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) gc[c][v] = 0.5 * (Gc[io + c] + Gc[in + c]);
        // the two liftings: c_P (q^com - q_own) (2/h) n_own + c_P (q^com - q_nbr) (2/h) n_nbr
        gc[d][v] += 0.5 * lift * sg * ((qcv[v] - qo[v]) - (qcv[v] - qn[v]));
      }
      double fv[5];
      vis3(qcv, gc, d, a, fv);
#pragma unroll
      for (int v = 0; v < 5; ++v) fc[v] -= fv[v];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double fl = 0.0;
      for (int m = 0; m < n; ++m) fl = fma(lw[m], F[d][v][line_pt<n>(d, j, m)], fl);
      tr[f][v][j] = fc[v] - fl;
    }
  }
  __syncthreads();
  for (int k = tid; k < Np; k += NT) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double R = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        int j, t;
        point_on_line<n>(k, d, &j, &t);
        double x = 0.0;
        for (int m = 0; m < n; ++m) x = fma(B.D[t][m], F[d][v][line_pt<n>(d, j, m)], x);
        x = fma(tr[2 * d][v][j], B.gL[t], x);
        x = fma(tr[2 * d + 1][v][j], B.gR[t], x);
        R = fma(-2.0 / a.h[d], x, R);
      }
      const size_t gi = ((size_t)v * nel + el) * Np + k;
      if constexpr (MODE == 0)
        outc[gi] = R;
      else
        outc[gi] = zero_v ? 0.0 : a.shift * a.V[gi] - (R - a.R0[gi]) / e;
    }
  }
}

// ---------------------------------------------------------------- SSPRK3 combination
// out = alpha A + beta (Bv + dt R)
__global__ void k3_combine(double* __restrict__ out, const double* __restrict__ A, const double* __restrict__ Bv,
                           const double* __restrict__ R, double alpha, double beta, double dt, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = alpha * A[i] + beta * fma(dt, R[i], Bv[i]);
}

// ---------------------------------------------------------------- dissipation diagnostics
// Per element: sum of w |J| (rho |u|^2 / 2), of w |J| S^d:S^d and of w |J| p div u, with the
// velocity gradient from the raw gradient of the element's solution polynomial.
template <int P>
__global__ void __launch_bounds__(C3<P>::NT) k3_dissip(const Args3 a, const Basis B, double* __restrict__ part) {
  using C = C3<P>;
  constexpr int n = C::n, Np = C::Np, NT = C::NT;
  __shared__ double q[5][Np];
  __shared__ double red[5][NT / 64];
  const int el = blockIdx.x, tid = threadIdx.x;
  const size_t nel = (size_t)a.nel;
  for (int k = tid; k < Np; k += NT)
#pragma unroll
    for (int v = 0; v < 5; ++v) q[v][k] = a.U[((size_t)v * nel + el) * Np + k];
  __syncthreads();
  const double J = a.h[0] * a.h[1] * a.h[2] / 8.0;
  double ek = 0.0, ss = 0.0, pd = 0.0, ps = 0.0, ds = 0.0;
  for (int k = tid; k < Np; k += NT) {
    double g[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int j, t;
      point_on_line<n>(k, d, &j, &t);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        double x = 0.0;
        for (int m = 0; m < n; ++m) x = fma(B.D[t][m], q[v][line_pt<n>(d, j, m)], x);
        g[d][v] = (2.0 / a.h[d]) * x;
      }
    }
    const double rho = q[0][k], ir = 1.0 / rho;
    const double u[3] = {q[1][k] * ir, q[2][k] * ir, q[3][k] * ir};
    double du[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) du[i][c] = (g[c][1 + i] - u[i] * g[c][0]) * ir;
    const double div = du[0][0] + du[1][1] + du[2][2];
    double s2 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double sd = 0.5 * (du[i][c] + du[c][i]) - ((i == c) ? div / 3.0 : 0.0);
        s2 = fma(sd, sd, s2);
      }
    const int ia = k % n, ib = (k / n) % n, ic = k / (n * n);
    const double w = J * B.w[ia] * B.w[ib] * B.w[ic];
    double qk[5] = {q[0][k], q[1][k], q[2][k], q[3][k], q[4][k]};
    ek = fma(w, 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]), ek);
    ss = fma(w, s2, ss);
    const double p = p3(qk, a.gamma);
    pd = fma(w, p * div, pd);
    ps = fma(w, p, ps);
    ds = fma(w, div, ds);
  }
  ek = wave_sum(ek);
  ss = wave_sum(ss);
  pd = wave_sum(pd);
  ps = wave_sum(ps);
  ds = wave_sum(ds);
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = ek;
    red[1][tid >> 6] = ss;
    red[2][tid >> 6] = pd;
    red[3][tid >> 6] = ps;
    red[4][tid >> 6] = ds;
  }
  __syncthreads();
  if (tid < 5) {
    double t = 0.0;
    for (int w = 0; w < NT / 64; ++w) t += red[tid][w];
    part[(size_t)el * 5 + tid] = t;
  }
}

// ---------------------------------------------------------------- launchers
static unsigned grid3(size_t n) { return (unsigned)std::min<size_t>((n + 255) / 256, 4096); }

template <int P, int FLUX>
static hipError_t res3_pf(const Args3& a, const Basis& B, int mode, bool visc, hipStream_t s) {
  using C = C3<P>;
  const dim3 g(a.nel), b(C::NT);
  if (mode == 0) {
    if (visc) {
      hipLaunchKernelGGL((k3_faces<P, 0, true>), g, b, 0, s, a, B);
      hipLaunchKernelGGL((k3_res<P, FLUX, 0, true>), g, b, 0, s, a, B);
    } else {
      hipLaunchKernelGGL((k3_faces<P, 0, false>), g, b, 0, s, a, B);
      hipLaunchKernelGGL((k3_res<P, FLUX, 0, false>), g, b, 0, s, a, B);
    }
  } else {
    if (visc) {
      hipLaunchKernelGGL((k3_faces<P, 1, true>), g, b, 0, s, a, B);
      hipLaunchKernelGGL((k3_res<P, FLUX, 1, true>), g, b, 0, s, a, B);
    } else {
      hipLaunchKernelGGL((k3_faces<P, 1, false>), g, b, 0, s, a, B);
      hipLaunchKernelGGL((k3_res<P, FLUX, 1, false>), g, b, 0, s, a, B);
    }
  }
  return hipGetLastError();
}

static Args3 args3(const fr3d_disc* d) {
  Args3 a{};
  a.nx = d->nx;
  a.ny = d->ny;
  a.nz = d->nz;
  a.nel = d->nel;
  for (int i = 0; i < 3; ++i) a.h[i] = d->h[i];
  a.gamma = d->gamma;
  a.rgas = d->rgas;
  a.mu = d->mu;
  a.cp_over_pr = d->gamma * d->rgas / (d->gamma - 1.0) / d->prandtl;
  return a;
}

size_t fr3d_trace_bytes(const fr3d_disc* d) {
  const size_t n2 = (size_t)d->n * d->n;
  const size_t t = (size_t)d->nel * 6 * 5 * n2 * sizeof(double);
  return ((t + 255) & ~(size_t)255) + ((d->mu != 0.0) ? ((3 * t + 255) & ~(size_t)255) : 0);
}

hipError_t launch_fr3d_residual(const fr3d_disc* d, int mode, const double* U, const double* V, const double* R0,
                                double shift, double eps, int eps_mode, const double* nrm2, double* out, void* work,
                                hipStream_t s) {
  Args3 a = args3(d);
  a.U = U;
  a.V = V;
  a.R0 = R0;
  a.out = out;
  a.shift = shift;
  a.eps = eps;
  a.eps_mode = eps_mode;
  a.nrm2 = nrm2;
  const size_t n2 = (size_t)d->n * d->n;
  const size_t t = (size_t)d->nel * 6 * 5 * n2 * sizeof(double);
  a.T = (double*)work;
  a.G = (d->mu != 0.0) ? (double*)((char*)work + ((t + 255) & ~(size_t)255)) : nullptr;
  const bool visc = d->mu != 0.0, roe = d->flux == FR_ROE;
  switch (d->p) {
    case 2: return roe ? res3_pf<2, 1>(a, d->basis, mode, visc, s) : res3_pf<2, 0>(a, d->basis, mode, visc, s);
    case 3: return roe ? res3_pf<3, 1>(a, d->basis, mode, visc, s) : res3_pf<3, 0>(a, d->basis, mode, visc, s);
    case 4: return roe ? res3_pf<4, 1>(a, d->basis, mode, visc, s) : res3_pf<4, 0>(a, d->basis, mode, visc, s);
  }
  return hipErrorInvalidValue;
}

// The plain residual (mode 0) on the elements elist[0 .. count) only: the first kernel
// writes their traces and face gradients, the second (unless faces_only) their R, reading
// the other elements' face data as the work buffer holds it.  With copies > 1, copy c
// (blockIdx.y) has its own state U + c ndof, output out + c ndof and face data at
// work + c face_stride bytes.
template <int P, int FLUX, bool VISC>
static hipError_t res3_subset(const Args3& a, const Basis& B, int count, int copies, bool faces_only,
                              hipStream_t s) {
  using C = C3<P>;
  const dim3 g(count, copies), b(C::NT);
  hipLaunchKernelGGL((k3_faces<P, 0, VISC>), g, b, 0, s, a, B);
  if (!faces_only) hipLaunchKernelGGL((k3_res<P, FLUX, 0, VISC>), g, b, 0, s, a, B);
  return hipGetLastError();
}

template <int P>
static hipError_t res3_subset_p(const fr3d_disc* d, const Args3& a, int count, int copies, bool faces_only,
                                hipStream_t s) {
  const bool roe = d->flux == FR_ROE, visc = d->mu != 0.0;
  if (visc)
    return roe ? res3_subset<P, 1, true>(a, d->basis, count, copies, faces_only, s)
               : res3_subset<P, 0, true>(a, d->basis, count, copies, faces_only, s);
  return roe ? res3_subset<P, 1, false>(a, d->basis, count, copies, faces_only, s)
             : res3_subset<P, 0, false>(a, d->basis, count, copies, faces_only, s);
}

hipError_t launch_fr3d_residual_subset(const fr3d_disc* d, const double* U, double* out, void* work,
                                       const int* elist, int count, int copies, size_t face_stride,
                                       bool faces_only, hipStream_t s) {
  if (count <= 0 || copies <= 0 || elist == nullptr) return hipErrorInvalidValue;
  Args3 a = args3(d);
  a.U = U;
  a.out = out;
  a.elist = elist;
  a.cs = copies > 1 ? d->ndof : 0;
  a.fs = copies > 1 ? face_stride : 0;
  const size_t n2 = (size_t)d->n * d->n;
  const size_t t = (size_t)d->nel * 6 * 5 * n2 * sizeof(double);
  a.T = (double*)work;
  a.G = (d->mu != 0.0) ? (double*)((char*)work + ((t + 255) & ~(size_t)255)) : nullptr;
  switch (d->p) {
    case 2: return res3_subset_p<2>(d, a, count, copies, faces_only, s);
    case 3: return res3_subset_p<3>(d, a, count, copies, faces_only, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fr3d_combine(double* out, const double* A, const double* Bv, const double* R, double alpha,
                               double beta, double dt, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k3_combine, dim3(grid3(n)), dim3(256), 0, s, out, A, Bv, R, alpha, beta, dt, n);
  return hipGetLastError();
}

hipError_t launch_fr3d_dissipation(const fr3d_disc* d, const double* U, double* part, hipStream_t s) {
  Args3 a = args3(d);
  a.U = U;
  switch (d->p) {
    case 2: hipLaunchKernelGGL((k3_dissip<2>), dim3(d->nel), dim3(C3<2>::NT), 0, s, a, d->basis, part); break;
    case 3: hipLaunchKernelGGL((k3_dissip<3>), dim3(d->nel), dim3(C3<3>::NT), 0, s, a, d->basis, part); break;
    case 4: hipLaunchKernelGGL((k3_dissip<4>), dim3(d->nel), dim3(C3<4>::NT), 0, s, a, d->basis, part); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace frjf
