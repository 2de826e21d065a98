// FR residual of the 2D Navier-Stokes equations with the BR1 common gradient
// (Section 2 viscous flux; Section 3: common state q^com = (q+ + q-)/2 and
// common gradient = mean of the two sides' corrected gradients), and its
// element-Jacobi block assembly.
//
// Kernel A (k_ns_grad): per element, the corrected gradient
//   dq/dxi~ = D q + (q^com - q)_{xi=-1} g_L' + (q^com - q)_{xi=+1} g_R'   (same in eta),
//   grad q = J^{-T} (dq/dxi~, dq/deta~),
// extrapolated to the four faces and written to a trace buffer
// grad[e][face][var][j][x|y].
// Kernel B (k_ns_res): the residual; the common gradient on a face averages
// the element's own face gradient and the neighbour's (from the buffer), so
// both sides of a face evaluate identical fluxes.
// Kernel C (k_ns_ejacobi): one workgroup per element, several finite-difference
// columns at once ("slots"); each column is a full element-local residual with
// every other element frozen.  A neighbour's face gradient on the shared face
// depends on this element only through the shared common state, linearly:
// grad_nbr = grad_nbr(base) + c_f (q^com - q^com(base)), with c_f computed
// from the neighbour's metrics.
//
// BR2 (Section 3, eq. com_grad_q and the lifting after it): an element's gradient on a
// face is the raw gradient of its solution polynomial (no corrections), extrapolated to
// the face, plus the lifting r = c_P (q^com - q_local) S_out / |J| of that face alone,
// c_P = (P+1)(P+2)/2 (the paper's g'(+-1)), S_out the outward area-weighted normal and
// |J| at the face point; the common gradient averages the two sides'.  The gradient
// inside the element stays the FR-corrected one.
// Boundaries (the eta = -1 side of row 0, the eta = +1 side of row ny-1; xi periodic):
//   far field: outside trace q_far, Riemann-solver flux, common state (q + q_far)/2;
//   wall (no slip, adiabatic): outside trace (rho, -rho u, -rho v, E - rho |u|^2), so the
//   common state has zero velocity and the inside internal energy; pressure flux
//   (0, p S_x, p S_y, 0); viscous flux at the common state, energy component zero.
// A boundary side's common gradient is its own face gradient.
//
// All three kernels run the same per-slot steps below; a slot is one element
// evaluation whose threads cover its solution points or face points.
#include <algorithm>
#include <cmath>

#include "internal.h"
#include "physics.h"

namespace frjf {

template <int P>
struct NS {
  static constexpr int n = P + 1, Np = n * n, Nb = 4 * Np;
  static constexpr int ST = (Np > 4 * n) ? Np : 4 * n;  // threads per slot
  static constexpr int SLOTS = 8;                        // slots per workgroup
  static constexpr int NT = ((ST * SLOTS + 63) / 64) * 64;
  static constexpr int LD = Nb + 1;
};

struct NSArgs {
  const double* U;
  const double* V;
  const double* R0;
  const double* B;
  double* out;
  double* grad;
  const double* nrm2;
  const int* skip;
  double eps, shift;
  int eps_mode;
  const double* nodes;
  int nx, ny, nel;
  int visc;      // FR_BR1 or FR_BR2
  int bcS, bcN;  // FR_BC_* of the eta = -1 side of row 0 and the eta = +1 side of row ny-1
  double qfar[4];
  Phys ph;
};

// boundary condition of face f (W, E, S, N) of an element in row ey (0: interior face)
__device__ __forceinline__ int face_bc(const NSArgs& a, int f, int ey) {
  if (f == 2 && ey == 0) return a.bcS;
  if (f == 3 && ey == a.ny - 1) return a.bcN;
  return FR_BC_PERIODIC;
}

// outside trace of a boundary face
__device__ __forceinline__ void ghost_state(int bc, const double qo[4], const double qfar[4], double qn[4]) {
  if (bc == FR_BC_WALL) {
    qn[0] = qo[0];
    qn[1] = -qo[1];
    qn[2] = -qo[2];
    qn[3] = qo[3] - (qo[1] * qo[1] + qo[2] * qo[2]) / qo[0];
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) qn[v] = qfar[v];
  }
}

// viscous flux f_v, g_v of Section 2 (2D) from q and its gradient
__device__ __forceinline__ void viscous_fluxes(const double q[4], const double qx[4], const double qy[4],
                                               const Phys& ph, double fv[4], double gv[4]) {
  const double ir = 1.0 / q[0];
  const double u = q[1] * ir, v = q[2] * ir;
  const double ux = (qx[1] - u * qx[0]) * ir, uy = (qy[1] - u * qy[0]) * ir;
  const double vx = (qx[2] - v * qx[0]) * ir, vy = (qy[2] - v * qy[0]) * ir;
  const double ke = 0.5 * (u * u + v * v);
  const double p = (ph.gamma - 1.0) * (q[3] - q[0] * ke);
  const double T = p * ir / ph.rgas;
  const double px = (ph.gamma - 1.0) * (qx[3] - ke * qx[0] - q[0] * (u * ux + v * vx));
  const double py = (ph.gamma - 1.0) * (qy[3] - ke * qy[0] - q[0] * (u * uy + v * vy));
  const double Tx = (px - ph.rgas * T * qx[0]) * ir / ph.rgas;
  const double Ty = (py - ph.rgas * T * qy[0]) * ir / ph.rgas;
  const double div = ux + vy;
  const double txx = ph.mu * (2.0 * ux - (2.0 / 3.0) * div);
  const double tyy = ph.mu * (2.0 * vy - (2.0 / 3.0) * div);
  const double txy = ph.mu * (uy + vx);
  const double kap = ph.mu * ph.cp_over_pr;
  fv[0] = 0.0;
  fv[1] = txx;
  fv[2] = txy;
  fv[3] = u * txx + v * txy + kap * Tx;
  gv[0] = 0.0;
  gv[1] = txy;
  gv[2] = tyy;
  gv[3] = u * txy + v * tyy + kap * Ty;
}

// Per-slot working set in LDS.
// The point fluxes F, G replace the gradient qx, qy in place: each point's fluxes
// need only that point's gradient, and the face gradients are taken before.
template <int P>
struct SlotData {
  static constexpr int n = P + 1, Np = n * n;
  double q[4][Np];
  union {
    struct {
      double qx[4][Np], qy[4][Np];
    };
    struct {
      double F[4][Np], G[4][Np];
    };
  };
  // the face jumps replace the solution traces: the thread of a face point reads
  // its traces before it writes that point's jumps
  union {
    double tr[4][4][n];
    double jmp[4][4][n];
  };
  double qc[4][4][n], gc[4][4][n][2];
};

template <int P>
using Slot = SlotData<P>;

// Per-element geometry and neighbour data in LDS.
template <int P>
struct ElemGeo {
  static constexpr int n = P + 1, Np = n * n;
  double met[Np][5];      // x_xi, x_eta, y_xi, y_eta, 1/|J|
  double S[4][2];         // area-weighted face normals (+xi / +eta)
  double Jf[4][n];        // |J| at the face points (BR2 lifting)
  double nb[4][4][n];     // neighbours' solution traces on the shared faces
  int nbr[4];             // neighbour element indices (-1 on a boundary side)
  int bc[4];              // FR_BC_* of each face
};

__device__ __forceinline__ void face_neighbour(int f, int ex, int ey, int nx, int ny, int* nex, int* ney) {
  *nex = ex;
  *ney = ey;
  if (f == 0) *nex = (ex == 0) ? nx - 1 : ex - 1;
  if (f == 1) *nex = (ex + 1 == nx) ? 0 : ex + 1;
  if (f == 2) *ney = (ey == 0) ? ny - 1 : ey - 1;
  if (f == 3) *ney = (ey + 1 == ny) ? 0 : ey + 1;
}

template <int MODE>
__device__ __forceinline__ double ns_state(const NSArgs& a, size_t gi, double e) {
  if constexpr (MODE == 0)
    return a.U[gi];
  else
    return fma(e, a.V[gi], a.U[gi]);
}

// geometry of element (ex, ey): metrics at the points, face normals, neighbour indices and
// the neighbours' solution traces (for state U or U + e V); t indexes the slot's threads
// V: compile-time variant, bit 0 = BR2 (else BR1), bit 1 = boundaries on the eta sides
// (else doubly periodic); the BR1 periodic kernels carry none of the other code.
enum { kVarBR2 = 1, kVarBnd = 2 };

template <int P, int MODE, int V>
__device__ void load_elem_geo(ElemGeo<P>& g, const NSArgs& a, const Basis& B, int ex, int ey, double e, int t,
                              int nthreads) {
  constexpr int n = P + 1, Np = n * n;
  const size_t nel = (size_t)a.nel;
  for (int k = t; k < Np; k += nthreads) {
    double c[8];
    load_corners(a.nodes, a.nx, ex, ey, c);
    const Metric m = bilinear_metric(c, B.x[k % n], B.x[k / n]);
    g.met[k][0] = m.xxi;
    g.met[k][1] = m.xeta;
    g.met[k][2] = m.yxi;
    g.met[k][3] = m.yeta;
    g.met[k][4] = 1.0 / m.J;
  }
  if (t < 4) {
    double Sx, Sy;
    const int bc = (V & kVarBnd) ? face_bc(a, t, ey) : FR_BC_PERIODIC;
    if (t == 0) xi_face_normal(a.nodes, a.nx, ex, ey, &Sx, &Sy);
    else if (t == 1) xi_face_normal(a.nodes, a.nx, (ex + 1 == a.nx) ? 0 : ex + 1, ey, &Sx, &Sy);
    else if (t == 2) eta_face_normal(a.nodes, a.nx, ex, ey, &Sx, &Sy);
    else eta_face_normal(a.nodes, a.nx, ex, (ey + 1 == a.ny && bc == FR_BC_PERIODIC) ? 0 : ey + 1, &Sx, &Sy);
    g.S[t][0] = Sx;
    g.S[t][1] = Sy;
    int nex, ney;
    face_neighbour(t, ex, ey, a.nx, a.ny, &nex, &ney);
    g.nbr[t] = bc == FR_BC_PERIODIC ? ney * a.nx + nex : -1;
    g.bc[t] = bc;
  }
  for (int idx = t; idx < 4 * n; idx += nthreads) {
    const int f = idx / n, j = idx % n;
    if constexpr ((V & kVarBR2) != 0) {
      double c[8];
      load_corners(a.nodes, a.nx, ex, ey, c);
      const double xi = f == 0 ? -1.0 : (f == 1 ? 1.0 : B.x[j]);
      const double eta = f == 2 ? -1.0 : (f == 3 ? 1.0 : B.x[j]);
      g.Jf[f][j] = bilinear_metric(c, xi, eta).J;
    }
    if ((V & kVarBnd) && face_bc(a, f, ey) != FR_BC_PERIODIC) continue;  // outside trace from the own one
    int nex, ney;
    face_neighbour(f, ex, ey, a.nx, a.ny, &nex, &ney);
    const size_t ne = (size_t)ney * a.nx + nex;
    const double* lo = (f == 0 || f == 2) ? B.lp : B.lm;
    double qn[4] = {0, 0, 0, 0};
    for (int c2 = 0; c2 < n; ++c2) {
      const int kk = (f < 2) ? j * n + c2 : c2 * n + j;
#pragma unroll
      for (int v = 0; v < 4; ++v) qn[v] = fma(lo[c2], ns_state<MODE>(a, ((size_t)v * nel + ne) * Np + kk, e), qn[v]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) g.nb[f][v][j] = qn[v];
  }
}

// step 2: own traces and common solution on the faces (a boundary side's outside trace
// from the own one)
template <int P, int V>
__device__ void slot_traces(Slot<P>& s, const ElemGeo<P>& g, const Basis& B, const double qfar[4], int t) {
  constexpr int n = P + 1;
  for (int idx = t; idx < 4 * n; idx += NS<P>::ST) {
    const int f = idx / n, j = idx % n;
    const double* lw = (f == 0 || f == 2) ? B.lm : B.lp;
    double qo[4], qn[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double x = 0.0;
      for (int c = 0; c < n; ++c) x = fma(lw[c], s.q[v][(f < 2) ? j * n + c : c * n + j], x);
      qo[v] = x;
    }
    if (!(V & kVarBnd) || g.bc[f] == FR_BC_PERIODIC) {
#pragma unroll
      for (int v = 0; v < 4; ++v) qn[v] = g.nb[f][v][j];
    } else {
      ghost_state(g.bc[f], qo, qfar, qn);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      s.tr[f][v][j] = qo[v];
      s.qc[f][v][j] = 0.5 * (qo[v] + qn[v]);
    }
  }
}

// step 3: corrected physical gradient at the solution points
template <int P>
__device__ void slot_gradient(Slot<P>& s, const ElemGeo<P>& g, const Basis& B, int t) {
  constexpr int n = P + 1, Np = n * n;
  for (int k = t; k < Np; k += NS<P>::ST) {
    const int ia = k % n, ib = k / n;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double dxi = 0.0, deta = 0.0;
      for (int c = 0; c < n; ++c) {
        dxi = fma(B.D[ia][c], s.q[v][ib * n + c], dxi);
        deta = fma(B.D[ib][c], s.q[v][c * n + ia], deta);
      }
      dxi = fma(s.qc[0][v][ib] - s.tr[0][v][ib], B.gL[ia], dxi);
      dxi = fma(s.qc[1][v][ib] - s.tr[1][v][ib], B.gR[ia], dxi);
      deta = fma(s.qc[2][v][ia] - s.tr[2][v][ia], B.gL[ib], deta);
      deta = fma(s.qc[3][v][ia] - s.tr[3][v][ia], B.gR[ib], deta);
      const double* m = g.met[k];
      s.qx[v][k] = (m[3] * dxi - m[2] * deta) * m[4];
      s.qy[v][k] = (-m[1] * dxi + m[0] * deta) * m[4];
    }
  }
}

// own face gradient of face point (f, j), variable v: BR1 the corrected gradient
// extrapolated; BR2 the raw gradient extrapolated plus the face's lifting
template <int P, int V>
__device__ __forceinline__ void own_face_gradient(const Slot<P>& s, const ElemGeo<P>& g, const Basis& B, int f, int j,
                                                  int v, double* gx, double* gy) {
  constexpr int n = P + 1;
  const double* lw = (f == 0 || f == 2) ? B.lm : B.lp;
  double x = 0.0, y = 0.0;
  if constexpr ((V & kVarBR2) == 0) {
    for (int c = 0; c < n; ++c) {
      const int kk = (f < 2) ? j * n + c : c * n + j;
      x = fma(lw[c], s.qx[v][kk], x);
      y = fma(lw[c], s.qy[v][kk], y);
    }
  } else {
    for (int c = 0; c < n; ++c) {
      const int kk = (f < 2) ? j * n + c : c * n + j;
      const int ia = kk % n, ib = kk / n;
      double dxi = 0.0, deta = 0.0;
      for (int d = 0; d < n; ++d) {
        dxi = fma(B.D[ia][d], s.q[v][ib * n + d], dxi);
        deta = fma(B.D[ib][d], s.q[v][d * n + ia], deta);
      }
      const double* m = g.met[kk];
      x = fma(lw[c], (m[3] * dxi - m[2] * deta) * m[4], x);
      y = fma(lw[c], (-m[1] * dxi + m[0] * deta) * m[4], y);
    }
    constexpr double cP = 0.5 * (P + 1) * (P + 2);
    const double sg = (f == 0 || f == 2) ? -1.0 : 1.0;  // outward normal = sg S
    const double lift = cP * (s.qc[f][v][j] - s.tr[f][v][j]) / g.Jf[f][j];
    x = fma(lift * sg, g.S[f][0], x);
    y = fma(lift * sg, g.S[f][1], y);
  }
  *gx = x;
  *gy = y;
}

// step 5: total transformed fluxes F, G at the solution points
template <int P>
__device__ void slot_fluxes(Slot<P>& s, const ElemGeo<P>& g, const Phys& ph, int t) {
  constexpr int n = P + 1, Np = n * n;
  for (int k = t; k < Np; k += NS<P>::ST) {
    double q[4], qx[4], qy[4], f[4], gg[4], fv[4], gv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      q[v] = s.q[v][k];
      qx[v] = s.qx[v][k];
      qy[v] = s.qy[v][k];
    }
    euler_fluxes(q, ph.gamma, f, gg);
    viscous_fluxes(q, qx, qy, ph, fv, gv);
    const double* m = g.met[k];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double ft = f[v] - fv[v], gt = gg[v] - gv[v];
      s.F[v][k] = m[3] * ft - m[1] * gt;
      s.G[v][k] = -m[2] * ft + m[0] * gt;
    }
  }
}

// common flux F^num (inviscid minus viscous, along S) of face point (f, j) from the own
// trace qo, the common state qc and the common gradient (gx, gy)
template <int FLUX, int V>
__device__ __forceinline__ void face_common_flux(int f, int bc, const double qo[4], const double qnb[4],
                                                 const double qfar[4], const double qc[4], const double gx[4],
                                                 const double gy[4], double Sx, double Sy, const Phys& ph,
                                                 double Fn[4]) {
  double Fi[4], fv[4], gv[4];
  if ((V & kVarBnd) && bc == FR_BC_WALL) {
    const double p = pressure_of(qo, ph.gamma);
    Fi[0] = 0.0;
    Fi[1] = p * Sx;
    Fi[2] = p * Sy;
    Fi[3] = 0.0;
  } else {
    const double* qn = ((V & kVarBnd) && bc == FR_BC_FARFIELD) ? qfar : qnb;
    if (f == 0 || f == 2)
      common_flux<FLUX>(qn, qo, Sx, Sy, ph.gamma, Fi);
    else
      common_flux<FLUX>(qo, qn, Sx, Sy, ph.gamma, Fi);
  }
  viscous_fluxes(qc, gx, gy, ph, fv, gv);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double vis = ((V & kVarBnd) && bc == FR_BC_WALL && v == 3) ? 0.0 : fv[v] * Sx + gv[v] * Sy;
    Fn[v] = Fi[v] - vis;
  }
}

// step 6: common fluxes and jumps on the faces (gc holds the common gradient)
template <int P, int FLUX, int V>
__device__ void slot_face_fluxes(Slot<P>& s, const ElemGeo<P>& g, const Basis& B, const Phys& ph,
                                 const double qfar[4], int t) {
  constexpr int n = P + 1;
  for (int idx = t; idx < 4 * n; idx += NS<P>::ST) {
    const int f = idx / n, j = idx % n;
    const double* lw = (f == 0 || f == 2) ? B.lm : B.lp;
    double qo[4], qn[4], Fl[4], qc[4], gx[4], gy[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      qo[v] = s.tr[f][v][j];
      qn[v] = g.nb[f][v][j];
      qc[v] = s.qc[f][v][j];
      gx[v] = s.gc[f][v][j][0];
      gy[v] = s.gc[f][v][j][1];
      double fl = 0.0;
      for (int c = 0; c < n; ++c) fl = fma(lw[c], (f < 2) ? s.F[v][j * n + c] : s.G[v][c * n + j], fl);
      Fl[v] = fl;
    }
    double Fn[4];
    face_common_flux<FLUX, V>(f, (V & kVarBnd) ? g.bc[f] : FR_BC_PERIODIC, qo, qn, qfar, qc, gx, gy, g.S[f][0],
                              g.S[f][1], ph, Fn);
#pragma unroll
    for (int v = 0; v < 4; ++v) s.jmp[f][v][j] = Fn[v] - Fl[v];
  }
}

// step 7: residual at point k, variable v
template <int P>
__device__ __forceinline__ double slot_residual(const Slot<P>& s, const ElemGeo<P>& g, const Basis& B, int k, int v) {
  constexpr int n = P + 1;
  const int ia = k % n, ib = k / n;
  double div = 0.0;
  for (int c = 0; c < n; ++c) {
    div = fma(B.D[ia][c], s.F[v][ib * n + c], div);
    div = fma(B.D[ib][c], s.G[v][c * n + ia], div);
  }
  div = fma(s.jmp[0][v][ib], B.gL[ia], div);
  div = fma(s.jmp[1][v][ib], B.gR[ia], div);
  div = fma(s.jmp[2][v][ia], B.gL[ib], div);
  div = fma(s.jmp[3][v][ia], B.gR[ib], div);
  return -div * g.met[k][4];
}

__device__ __forceinline__ size_t grad_index(int el, int f, int v, int j, int n) {
  return ((((size_t)el * 4 + f) * 4 + v) * n + j) * 2;
}

// ---------------------------------------------------------------- kernel A: face gradient traces
template <int P, int MODE, int V>
__global__ void __launch_bounds__(NS<P>::NT) k_ns_grad(const NSArgs a, const Basis B) {
  using C = NS<P>;
  constexpr int n = C::n, Np = C::Np, ST = C::ST, SL = C::SLOTS;
  __shared__ Slot<P> S[SL];
  __shared__ ElemGeo<P> Gm[SL];
  if (MODE != 0 && a.skip != nullptr && *a.skip) return;
  const int sl = threadIdx.x / ST, t = threadIdx.x % ST;
  const int el = blockIdx.x * SL + sl;
  const bool live = sl < SL && el < a.nel;
  const size_t nel = (size_t)a.nel;
  double e = 0.0;
  if constexpr (MODE != 0) {
    if (a.eps_mode == FR_EPS_RMS) {
      const double n2 = *a.nrm2;
      e = (n2 > 0.0) ? a.eps / sqrt(n2 / (double)(4 * nel * Np)) : 0.0;
    } else {
      e = a.eps;
    }
  }
  const int ex = live ? el % a.nx : 0, ey = live ? el / a.nx : 0;
  if (live) {
    load_elem_geo<P, MODE, V>(Gm[sl], a, B, ex, ey, e, t, ST);
    for (int k = t; k < Np; k += ST)
#pragma unroll
      for (int v = 0; v < 4; ++v) S[sl].q[v][k] = ns_state<MODE>(a, ((size_t)v * nel + el) * Np + k, e);
  }
  __syncthreads();
  if (live) slot_traces<P, V>(S[sl], Gm[sl], B, a.qfar, t);
  __syncthreads();
  if (live) slot_gradient<P>(S[sl], Gm[sl], B, t);
  __syncthreads();
  if (live)
    for (int idx = t; idx < 4 * n; idx += ST) {
      const int f = idx / n, j = idx % n;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double gx, gy;
        own_face_gradient<P, V>(S[sl], Gm[sl], B, f, j, v, &gx, &gy);
        const size_t gi = grad_index(el, f, v, j, n);
        a.grad[gi] = gx;
        a.grad[gi + 1] = gy;
      }
    }
}

// ---------------------------------------------------------------- kernel B: residual
template <int P, int FLUX, int MODE, int V>
__global__ void __launch_bounds__(NS<P>::NT) k_ns_res(const NSArgs a, const Basis B) {
  using C = NS<P>;
  constexpr int n = C::n, Np = C::Np, ST = C::ST, SL = C::SLOTS;
  __shared__ Slot<P> S[SL];
  __shared__ ElemGeo<P> Gm[SL];
  if (MODE != 0 && a.skip != nullptr && *a.skip) return;
  const int sl = threadIdx.x / ST, t = threadIdx.x % ST;
  const int el = blockIdx.x * SL + sl;
  const bool live = sl < SL && el < a.nel;
  const size_t nel = (size_t)a.nel;
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
  const int ex = live ? el % a.nx : 0, ey = live ? el / a.nx : 0;
  if (live) {
    load_elem_geo<P, MODE, V>(Gm[sl], a, B, ex, ey, e, t, ST);
    for (int k = t; k < Np; k += ST)
#pragma unroll
      for (int v = 0; v < 4; ++v) S[sl].q[v][k] = ns_state<MODE>(a, ((size_t)v * nel + el) * Np + k, e);
  }
  __syncthreads();
  if (live) slot_traces<P, V>(S[sl], Gm[sl], B, a.qfar, t);
  __syncthreads();
  if (live) slot_gradient<P>(S[sl], Gm[sl], B, t);
  __syncthreads();
  if (live)
    for (int idx = t; idx < 4 * n; idx += ST) {
      const int f = idx / n, j = idx % n;
      const int o = f ^ 1;  // the neighbour's face opposite to f
      const int ne = Gm[sl].nbr[f];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double gx, gy;
        own_face_gradient<P, V>(S[sl], Gm[sl], B, f, j, v, &gx, &gy);
        if ((V & kVarBnd) && ne < 0) {  // boundary side: its own face gradient
          S[sl].gc[f][v][j][0] = gx;
          S[sl].gc[f][v][j][1] = gy;
        } else {
          const size_t gi = grad_index(ne, o, v, j, n);
          S[sl].gc[f][v][j][0] = 0.5 * (gx + a.grad[gi]);
          S[sl].gc[f][v][j][1] = 0.5 * (gy + a.grad[gi + 1]);
        }
      }
    }
  __syncthreads();
  if (live) slot_fluxes<P>(S[sl], Gm[sl], a.ph, t);
  __syncthreads();
  if (live) slot_face_fluxes<P, FLUX, V>(S[sl], Gm[sl], B, a.ph, a.qfar, t);
  __syncthreads();
  if (live)
    for (int k = t; k < Np; k += ST)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double R = slot_residual<P>(S[sl], Gm[sl], B, k, v);
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

// ---------------------------------------------------------------- kernel C: element-Jacobi blocks

template <int P, int FLUX, typename T, int V>
__global__ void __launch_bounds__(NS<P>::NT) k_ns_ejacobi(const NSArgs a, const Basis B, void* outp) {
  using C = NS<P>;
  constexpr int n = C::n, Np = C::Np, Nb = C::Nb, ST = C::ST, SL = C::SLOTS, NT = C::NT, LD = C::LD;
  __shared__ Slot<P> S[SL];
  __shared__ ElemGeo<P> Gm;
  __shared__ double gnb[4][4][P + 1][2];  // neighbours' face gradients on the shared faces
  __shared__ double q0[4][Np], R0[4][Np], qc0[4][4][n], cg[4][n][2];
  __shared__ T A[Nb * LD];  // the block, column-major, padded leading dimension
  const int tid = threadIdx.x;
  const int sl = tid / ST, t = tid % ST;
  const int el = blockIdx.x;
  const int ex = el % a.nx, ey = el / a.nx;
  const size_t nel = (size_t)a.nel;

  if (tid < ST) load_elem_geo<P, 0, V>(Gm, a, B, ex, ey, 0.0, tid, ST);
  for (int k = tid; k < Np; k += NT)
#pragma unroll
    for (int v = 0; v < 4; ++v) q0[v][k] = a.U[((size_t)v * nel + el) * Np + k];
  __syncthreads();
  // neighbours' base face gradients on the shared faces, and the coefficients c_f of their
  // dependence on the shared common state (from the neighbour's metrics)
  for (int idx = tid; idx < 4 * n; idx += NT) {
    const int f = idx / n, j = idx % n;
    const int o = f ^ 1;
    const int ne = Gm.nbr[f];
    if ((V & kVarBnd) && ne < 0) continue;  // boundary side: no neighbour
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const size_t gi = grad_index(ne, o, v, j, n);
      gnb[f][v][j][0] = a.grad[gi];
      gnb[f][v][j][1] = a.grad[gi + 1];
    }
    double c8[8];
    load_corners(a.nodes, a.nx, ne % a.nx, ne / a.nx, c8);
    double cx = 0.0, cy = 0.0;
    if constexpr ((V & kVarBR2) != 0) {
      // the neighbour's lifting c_P (q^com - q_nbr) S_out,nbr / |J_nbr| on the shared face;
      // its outward normal there is +S on this element's W and S faces, -S on E and N
      const double xi = o == 0 ? -1.0 : (o == 1 ? 1.0 : B.x[j]);
      const double eta = o == 2 ? -1.0 : (o == 3 ? 1.0 : B.x[j]);
      const double Jn = bilinear_metric(c8, xi, eta).J;
      const double sg = (f == 0 || f == 2) ? 1.0 : -1.0;
      constexpr double cP = 0.5 * (P + 1) * (P + 2);
      cx = cP * sg * Gm.S[f][0] / Jn;
      cy = cP * sg * Gm.S[f][1] / Jn;
    } else {
      // neighbour face o: E(1) -> its xi = +1 lifted with g_R'; W(0) -> xi = -1 with g_L'
      // (likewise N(3)/S(2) in eta); the neighbour's face values extrapolate with l(+-1)
      for (int c = 0; c < n; ++c) {
        const bool xi_dir = (o < 2);
        const int ia = xi_dir ? c : j, ib = xi_dir ? j : c;
        const Metric m = bilinear_metric(c8, B.x[ia], B.x[ib]);
        const double lift = (o == 0 || o == 2) ? B.gL[c] : B.gR[c];
        const double ext = (o == 0 || o == 2) ? B.lm[c] : B.lp[c];
        if (xi_dir) {
          cx += ext * lift * m.yeta / m.J;
          cy += ext * lift * (-m.xeta) / m.J;
        } else {
          cx += ext * lift * (-m.yxi) / m.J;
          cy += ext * lift * m.xxi / m.J;
        }
      }
    }
    cg[f][j][0] = cx;
    cg[f][j][1] = cy;
  }
  __syncthreads();

  // columns in batches of SL; batch -1 is the base evaluation (slot 0)
  for (int j0 = -SL; j0 < Nb; j0 += SL) {
    const int jc = j0 + sl;                       // column of this slot (base if j0 < 0 && sl == 0)
    const bool base = (j0 < 0);
    const bool active = sl < SL && (base ? sl == 0 : jc < Nb);
    const int pv = active && !base ? jc / Np : -1, pk = active && !base ? jc % Np : -1;
    double delta = 0.0;
    if (pv >= 0) delta = 1e-8 * fmax(1.0, fabs(q0[pv][pk]));
    if (active)
      for (int k = t; k < Np; k += ST)
#pragma unroll
        for (int v = 0; v < 4; ++v) S[sl].q[v][k] = q0[v][k] + ((v == pv && k == pk) ? delta : 0.0);
    __syncthreads();
    if (active) slot_traces<P, V>(S[sl], Gm, B, a.qfar, t);
    __syncthreads();
    if (active) slot_gradient<P>(S[sl], Gm, B, t);
    if (base && active)
      for (int idx = t; idx < 4 * n; idx += ST) {
        const int f = idx / n, jj = idx % n;
#pragma unroll
        for (int v = 0; v < 4; ++v) qc0[f][v][jj] = S[0].qc[f][v][jj];
      }
    __syncthreads();
    if (active)
      for (int idx = t; idx < 4 * n; idx += ST) {
        const int f = idx / n, jj = idx % n;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double gx, gy;
          own_face_gradient<P, V>(S[sl], Gm, B, f, jj, v, &gx, &gy);
          if ((V & kVarBnd) && Gm.nbr[f] < 0) {  // boundary side: its own face gradient
            S[sl].gc[f][v][jj][0] = gx;
            S[sl].gc[f][v][jj][1] = gy;
            continue;
          }
          const double dqc = S[sl].qc[f][v][jj] - qc0[f][v][jj];
          const double nx_ = gnb[f][v][jj][0] + cg[f][jj][0] * dqc;
          const double ny_ = gnb[f][v][jj][1] + cg[f][jj][1] * dqc;
          S[sl].gc[f][v][jj][0] = 0.5 * (gx + nx_);
          S[sl].gc[f][v][jj][1] = 0.5 * (gy + ny_);
        }
      }
    __syncthreads();
    if (active) slot_fluxes<P>(S[sl], Gm, a.ph, t);
    __syncthreads();
    if (active) slot_face_fluxes<P, FLUX, V>(S[sl], Gm, B, a.ph, a.qfar, t);
    __syncthreads();
    if (active)
      for (int k = t; k < Np; k += ST)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double R = slot_residual<P>(S[sl], Gm, B, k, v);
          if (base) {
            R0[v][k] = R;
          } else {
            double val = -(R - R0[v][k]) / delta;
            if (v * Np + k == jc) val += a.shift;
            A[jc * LD + v * Np + k] = (T)val;
          }
        }
    __syncthreads();
  }
  T* out = reinterpret_cast<T*>(outp) + (size_t)el * Nb * Nb;
  for (int idx = tid; idx < Nb * Nb; idx += NT) out[idx] = A[(idx / Nb) * LD + idx % Nb];
}

// ---------------------------------------------------------------- wall momentum flux
// One slot per element of row 0 (its eta = -1 side a wall): the element's own steps up to
// its face gradients, then sum_j w_j F^num(j) of the momentum on the wall face (S per unit
// reference length) into part[2 ex], part[2 ex + 1].  A boundary side needs no neighbour
// gradient, so no gradient traces are formed.
template <int P, int FLUX, int V>
__global__ void __launch_bounds__(NS<P>::NT) k_ns_wall_flux(const NSArgs a, const Basis B, double* part) {
  using C = NS<P>;
  constexpr int n = C::n, Np = C::Np, ST = C::ST, SL = C::SLOTS;
  __shared__ Slot<P> S[SL];
  __shared__ ElemGeo<P> Gm[SL];
  const int sl = threadIdx.x / ST, t = threadIdx.x % ST;
  const int el = blockIdx.x * SL + sl;  // row 0: element index = ex
  const bool live = sl < SL && el < a.nx;
  const size_t nel = (size_t)a.nel;
  if (live) {
    load_elem_geo<P, 0, V>(Gm[sl], a, B, el, 0, 0.0, t, ST);
    for (int k = t; k < Np; k += ST)
#pragma unroll
      for (int v = 0; v < 4; ++v) S[sl].q[v][k] = a.U[((size_t)v * nel + el) * Np + k];
  }
  __syncthreads();
  if (live) slot_traces<P, V>(S[sl], Gm[sl], B, a.qfar, t);
  __syncthreads();
  if (live) slot_gradient<P>(S[sl], Gm[sl], B, t);
  __syncthreads();
  if (live && t == 0) {
    double fx = 0.0, fy = 0.0;
    for (int j = 0; j < n; ++j) {
      double qo[4], qc[4], gx[4], gy[4], Fn[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        qo[v] = S[sl].tr[2][v][j];
        qc[v] = S[sl].qc[2][v][j];
        own_face_gradient<P, V>(S[sl], Gm[sl], B, 2, j, v, &gx[v], &gy[v]);
      }
      face_common_flux<FLUX, V>(2, FR_BC_WALL, qo, qo, a.qfar, qc, gx, gy, Gm[sl].S[2][0], Gm[sl].S[2][1], a.ph, Fn);
      fx = fma(B.w[j], Fn[1], fx);
      fy = fma(B.w[j], Fn[2], fy);
    }
    part[2 * el] = fx;
    part[2 * el + 1] = fy;
  }
}

// ---------------------------------------------------------------- launchers
static NSArgs ns_args(const fr_disc* d, const ResArgs& r) {
  NSArgs a{};
  a.U = r.U;
  a.V = r.V;
  a.R0 = r.R0;
  a.B = r.B;
  a.out = r.out;
  a.grad = r.grad;
  a.nrm2 = r.nrm2;
  a.skip = r.skip;
  a.eps = r.eps;
  a.shift = r.shift;
  a.eps_mode = r.eps_mode;
  a.nodes = d->nodes;
  a.nx = d->nx;
  a.ny = d->ny;
  a.nel = d->nel;
  a.visc = d->visc;
  a.bcS = d->bc_south;
  a.bcN = d->bc_north;
  for (int v = 0; v < 4; ++v) a.qfar[v] = d->qfar[v];
  a.ph = d->phys;
  return a;
}

template <int P, int FLUX, int V>
static hipError_t ns_res_pfv(const fr_disc* d, int mode, const NSArgs& a, hipStream_t s) {
  using C = NS<P>;
  dim3 grid((d->nel + C::SLOTS - 1) / C::SLOTS), block(C::NT);
  if (mode == 0) {
    hipLaunchKernelGGL((k_ns_grad<P, 0, V>), grid, block, 0, s, a, d->basis);
    hipLaunchKernelGGL((k_ns_res<P, FLUX, 0, V>), grid, block, 0, s, a, d->basis);
  } else if (mode == 1) {
    hipLaunchKernelGGL((k_ns_grad<P, 1, V>), grid, block, 0, s, a, d->basis);
    hipLaunchKernelGGL((k_ns_res<P, FLUX, 1, V>), grid, block, 0, s, a, d->basis);
  } else {
    hipLaunchKernelGGL((k_ns_grad<P, 2, V>), grid, block, 0, s, a, d->basis);
    hipLaunchKernelGGL((k_ns_res<P, FLUX, 2, V>), grid, block, 0, s, a, d->basis);
  }
  return hipGetLastError();
}

// the compile-time variant of a disc: BR2 and / or boundaries
static int ns_variant(const fr_disc* d) {
  return (d->visc == FR_BR2 ? kVarBR2 : 0) |
         ((d->bc_south != FR_BC_PERIODIC || d->bc_north != FR_BC_PERIODIC) ? kVarBnd : 0);
}

template <int P, int FLUX>
static hipError_t ns_res_pf(const fr_disc* d, int mode, const NSArgs& a, hipStream_t s) {
  switch (ns_variant(d)) {
    case 0: return ns_res_pfv<P, FLUX, 0>(d, mode, a, s);
    case 1: return ns_res_pfv<P, FLUX, 1>(d, mode, a, s);
    case 2: return ns_res_pfv<P, FLUX, 2>(d, mode, a, s);
    default: return ns_res_pfv<P, FLUX, 3>(d, mode, a, s);
  }
}

template <int P>
static hipError_t ns_res_p(const fr_disc* d, int mode, const NSArgs& a, hipStream_t s) {
  return d->flux == FR_ROE ? ns_res_pf<P, 1>(d, mode, a, s) : ns_res_pf<P, 0>(d, mode, a, s);
}

hipError_t launch_ns_residual(const fr_disc* d, int mode, const ResArgs& r, hipStream_t s) {
  if (r.grad == nullptr) return hipErrorInvalidValue;
  const NSArgs a = ns_args(d, r);
  switch (d->p) {
    case 2: return ns_res_p<2>(d, mode, a, s);
    case 3: return ns_res_p<3>(d, mode, a, s);
    case 4: return ns_res_p<4>(d, mode, a, s);
  }
  return hipErrorInvalidValue;
}

template <int P, int FLUX>
static hipError_t ns_wall_pf(const fr_disc* d, const NSArgs& a, double* part, hipStream_t s) {
  using C = NS<P>;
  const dim3 grid((d->nx + C::SLOTS - 1) / C::SLOTS), block(C::NT);
  if (d->visc == FR_BR2)
    hipLaunchKernelGGL((k_ns_wall_flux<P, FLUX, kVarBnd | kVarBR2>), grid, block, 0, s, a, d->basis, part);
  else
    hipLaunchKernelGGL((k_ns_wall_flux<P, FLUX, kVarBnd>), grid, block, 0, s, a, d->basis, part);
  return hipGetLastError();
}

hipError_t launch_ns_wall_flux(const fr_disc* d, const double* U, double* part, hipStream_t s) {
  ResArgs r{};
  r.U = U;
  const NSArgs a = ns_args(d, r);
  const bool roe = d->flux == FR_ROE;
  switch (d->p) {
    case 2: return roe ? ns_wall_pf<2, 1>(d, a, part, s) : ns_wall_pf<2, 0>(d, a, part, s);
    case 3: return roe ? ns_wall_pf<3, 1>(d, a, part, s) : ns_wall_pf<3, 0>(d, a, part, s);
    case 4: return roe ? ns_wall_pf<4, 1>(d, a, part, s) : ns_wall_pf<4, 0>(d, a, part, s);
  }
  return hipErrorInvalidValue;
}

template <int P, int FLUX, int V>
static hipError_t ns_asm_pfv(const fr_disc* d, const NSArgs& a, void* out, int precision, int invert, hipStream_t s) {
  using C = NS<P>;
  dim3 grid((d->nel + C::SLOTS - 1) / C::SLOTS), block(C::NT);
  hipLaunchKernelGGL((k_ns_grad<P, 0, V>), grid, block, 0, s, a, d->basis);
  dim3 g2(d->nel);
  if (precision == FR_F32) {
    // FP32: the FP64 blocks rounded on the way out, then inverted in place on MFMA
    if (!invert) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_ns_ejacobi<P, FLUX, float, V>), g2, block, 0, s, a, d->basis, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_gj_mfma_f32(4 * (P + 1) * (P + 1), static_cast<float*>(out), d->nel, s);
  } else {
    // FP64: the raw blocks, then their inverses in place
    hipLaunchKernelGGL((k_ns_ejacobi<P, FLUX, double, V>), g2, block, 0, s, a, d->basis, out);
    if (invert) {
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      return launch_invert_f64(4 * (P + 1) * (P + 1), static_cast<double*>(out), d->nel, s);
    }
  }
  return hipGetLastError();
}

template <int P, int FLUX>
static hipError_t ns_asm_pf(const fr_disc* d, const NSArgs& a, void* out, int precision, int invert, hipStream_t s) {
  switch (ns_variant(d)) {
    case 0: return ns_asm_pfv<P, FLUX, 0>(d, a, out, precision, invert, s);
    case 1: return ns_asm_pfv<P, FLUX, 1>(d, a, out, precision, invert, s);
    case 2: return ns_asm_pfv<P, FLUX, 2>(d, a, out, precision, invert, s);
    default: return ns_asm_pfv<P, FLUX, 3>(d, a, out, precision, invert, s);
  }
}

hipError_t launch_ns_ejacobi_assemble(const fr_disc* d, const double* U, double shift, void* out, int precision,
                                      int invert, double* grad, hipStream_t s) {
  if (grad == nullptr) return hipErrorInvalidValue;
  ResArgs r{};
  r.U = U;
  r.grad = grad;
  r.shift = shift;
  NSArgs a = ns_args(d, r);
  const bool roe = d->flux == FR_ROE;
  switch (d->p) {
    case 2: return roe ? ns_asm_pf<2, 1>(d, a, out, precision, invert, s) : ns_asm_pf<2, 0>(d, a, out, precision, invert, s);
    case 3: return roe ? ns_asm_pf<3, 1>(d, a, out, precision, invert, s) : ns_asm_pf<3, 0>(d, a, out, precision, invert, s);
    case 4: return roe ? ns_asm_pf<4, 1>(d, a, out, precision, invert, s) : ns_asm_pf<4, 0>(d, a, out, precision, invert, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace frjf
