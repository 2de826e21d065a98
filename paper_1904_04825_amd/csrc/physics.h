// Device-side physics of the 2D Euler / Navier-Stokes equations (Section 2)
// and the inviscid common fluxes used at element interfaces (Section 3).
#pragma once
#include <hip/hip_runtime.h>

namespace frjf {

__device__ __forceinline__ double pressure_of(const double q[4], double gam) {
  return (gam - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0]);
}

// f (x-flux) and g (y-flux) of q = (rho, rho u, rho v, E).
__device__ __forceinline__ void euler_fluxes(const double q[4], double gam, double f[4], double g[4]) {
  const double ir = 1.0 / q[0];
  const double u = q[1] * ir, v = q[2] * ir;
  const double p = (gam - 1.0) * (q[3] - 0.5 * (q[1] * u + q[2] * v));
  f[0] = q[1];
  f[1] = q[1] * u + p;
  f[2] = q[2] * u;
  f[3] = u * (q[3] + p);
  g[0] = q[2];
  g[1] = q[1] * v;
  g[2] = q[2] * v + p;
  g[3] = v * (q[3] + p);
}

// Normal flux along the unit normal (nx, ny); also returns |u_n| + c.
__device__ __forceinline__ void normal_flux_speed(const double q[4], double nx, double ny, double gam,
                                                  double fn[4], double* speed) {
  const double ir = 1.0 / q[0];
  const double u = q[1] * ir, v = q[2] * ir;
  const double p = (gam - 1.0) * (q[3] - 0.5 * (q[1] * u + q[2] * v));
  const double un = u * nx + v * ny;
  fn[0] = q[0] * un;
  fn[1] = q[1] * un + p * nx;
  fn[2] = q[2] * un + p * ny;
  fn[3] = (q[3] + p) * un;
  *speed = fabs(un) + sqrt(gam * p * ir);
}

// Rusanov (local Lax-Friedrichs): (fL + fR)/2 - lambda (qR - qL)/2, lambda = max |u_n| + c.
// S is the area-weighted normal; returns |S| f^com (eq. norm_num_f).
__device__ __forceinline__ void rusanov_flux(const double qL[4], const double qR[4], double Sx, double Sy,
                                             double gam, double out[4]) {
  const double mag = sqrt(Sx * Sx + Sy * Sy);
  const double nx = Sx / mag, ny = Sy / mag;
  double fL[4], fR[4], sL, sR;
  normal_flux_speed(qL, nx, ny, gam, fL, &sL);
  normal_flux_speed(qR, nx, ny, gam, fR, &sR);
  const double lam = fmax(sL, sR);
#pragma unroll
  for (int v = 0; v < 4; ++v) out[v] = mag * (0.5 * (fL[v] + fR[v]) - 0.5 * lam * (qR[v] - qL[v]));
}

// Roe flux (eq. invis_com): (fL + fR)/2 - R|Lambda|R^{-1}(qR - qL)/2 at the Roe average,
// expressed with the four characteristic wave strengths; no entropy fix.
__device__ __forceinline__ void roe_flux(const double qL[4], const double qR[4], double Sx, double Sy,
                                         double gam, double out[4]) {
  const double mag = sqrt(Sx * Sx + Sy * Sy);
  const double nx = Sx / mag, ny = Sy / mag;
  double fL[4], fR[4], sL, sR;
  normal_flux_speed(qL, nx, ny, gam, fL, &sL);
  normal_flux_speed(qR, nx, ny, gam, fR, &sR);
  const double rL = qL[0], rR = qR[0];
  const double uL = qL[1] / rL, vL = qL[2] / rL, uR = qR[1] / rR, vR = qR[2] / rR;
  const double pL = pressure_of(qL, gam), pR = pressure_of(qR, gam);
  const double HL = (qL[3] + pL) / rL, HR = (qR[3] + pR) / rR;
  const double sl = sqrt(rL), sr = sqrt(rR), isum = 1.0 / (sl + sr);
  const double rho = sl * sr;
  const double u = (sl * uL + sr * uR) * isum;
  const double v = (sl * vL + sr * vR) * isum;
  const double H = (sl * HL + sr * HR) * isum;
  const double q2 = u * u + v * v;
  const double c2 = (gam - 1.0) * (H - 0.5 * q2);
  const double c = sqrt(c2);
  const double un = u * nx + v * ny;
  const double ut = -u * ny + v * nx;
  const double dr = rR - rL, dp = pR - pL;
  const double dun = (uR - uL) * nx + (vR - vL) * ny;
  const double dut = -(uR - uL) * ny + (vR - vL) * nx;
  const double a1 = fabs(un - c) * (dp - rho * c * dun) / (2.0 * c2);
  const double a2 = fabs(un) * (dr - dp / c2);
  const double a3 = fabs(un) * rho * dut;
  const double a4 = fabs(un + c) * (dp + rho * c * dun) / (2.0 * c2);
  double d[4];
  d[0] = a1 + a2 + a4;
  d[1] = a1 * (u - c * nx) + a2 * u - a3 * ny + a4 * (u + c * nx);
  d[2] = a1 * (v - c * ny) + a2 * v + a3 * nx + a4 * (v + c * ny);
  d[3] = a1 * (H - un * c) + a2 * 0.5 * q2 + a3 * ut + a4 * (H + un * c);
#pragma unroll
  for (int k = 0; k < 4; ++k) out[k] = mag * (0.5 * (fL[k] + fR[k]) - 0.5 * d[k]);
}

// Rusanov flux with the area-weighted normal S directly: |S| f^com =
// (f_S(qL) + f_S(qR))/2 - Lambda (qR - qL)/2, f_S = f S_x + g S_y,
// Lambda = max(|u.S| + c|S|) of the two sides (no normalisation of S needed).
__device__ __forceinline__ void rusanov_flux_S(const double qL[4], const double qR[4], double Sx, double Sy,
                                               double magS, double gam, double out[4]) {
  double lam = 0.0;
  double fs[2][4];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const double* q = side ? qR : qL;
    const double ir = 1.0 / q[0];
    const double u = q[1] * ir, v = q[2] * ir;
    const double p = (gam - 1.0) * (q[3] - 0.5 * (q[1] * u + q[2] * v));
    const double uS = u * Sx + v * Sy;
    fs[side][0] = q[0] * uS;
    fs[side][1] = q[1] * uS + p * Sx;
    fs[side][2] = q[2] * uS + p * Sy;
    fs[side][3] = (q[3] + p) * uS;
    lam = fmax(lam, fabs(uS) + sqrt(gam * p * ir) * magS);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) out[v] = 0.5 * (fs[0][v] + fs[1][v]) - 0.5 * lam * (qR[v] - qL[v]);
}

template <int FLUX>
__device__ __forceinline__ void common_flux(const double qL[4], const double qR[4], double Sx, double Sy,
                                            double gam, double out[4]) {
  if constexpr (FLUX == 0)
    rusanov_flux(qL, qR, Sx, Sy, gam, out);
  else
    roe_flux(qL, qR, Sx, Sy, gam, out);
}

// Bilinear map metrics at reference point (xi, eta) from the corners
// c00, c10, c01, c11 (x then y).
struct Metric {
  double xxi, xeta, yxi, yeta, J;
};
__device__ __forceinline__ Metric bilinear_metric(const double c[8], double xi, double eta) {
  // c = {x00, y00, x10, y10, x01, y01, x11, y11}
  Metric m;
  m.xxi = 0.25 * ((c[2] - c[0]) * (1.0 - eta) + (c[6] - c[4]) * (1.0 + eta));
  m.yxi = 0.25 * ((c[3] - c[1]) * (1.0 - eta) + (c[7] - c[5]) * (1.0 + eta));
  m.xeta = 0.25 * ((c[4] - c[0]) * (1.0 - xi) + (c[6] - c[2]) * (1.0 + xi));
  m.yeta = 0.25 * ((c[5] - c[1]) * (1.0 - xi) + (c[7] - c[3]) * (1.0 + xi));
  m.J = m.xxi * m.yeta - m.xeta * m.yxi;
  return m;
}

__device__ __forceinline__ void load_corners(const double* __restrict__ nodes, int nx, int ex, int ey,
                                             double c[8]) {
  const int stride = nx + 1;
  const double* p00 = nodes + 2 * (ey * stride + ex);
  const double* p01 = nodes + 2 * ((ey + 1) * stride + ex);
  c[0] = p00[0];
  c[1] = p00[1];
  c[2] = p00[2];
  c[3] = p00[3];
  c[4] = p01[0];
  c[5] = p01[1];
  c[6] = p01[2];
  c[7] = p01[3];
}

// Area-weighted normals of the four faces of element (ex, ey), computed from the
// two end nodes of the shared edge, with the periodic edge column / row taken
// modulo the mesh so both neighbours see identical values.
// xi-faces: S = (y_eta, -x_eta) = ((y_t - y_b)/2, -(x_t - x_b)/2);
// eta-faces: S = (-y_xi, x_xi) = (-(y_r - y_l)/2, (x_r - x_l)/2).
__device__ __forceinline__ void xi_face_normal(const double* __restrict__ nodes, int nx, int i, int ey,
                                               double* Sx, double* Sy) {
  const int stride = nx + 1;
  const double* b = nodes + 2 * (ey * stride + i);
  const double* t = nodes + 2 * ((ey + 1) * stride + i);
  *Sx = 0.5 * (t[1] - b[1]);
  *Sy = -0.5 * (t[0] - b[0]);
}
__device__ __forceinline__ void eta_face_normal(const double* __restrict__ nodes, int nx, int ex, int j,
                                                double* Sx, double* Sy) {
  const int stride = nx + 1;
  const double* l = nodes + 2 * (j * stride + ex);
  const double* r = l + 2;
  *Sx = -0.5 * (r[1] - l[1]);
  *Sy = 0.5 * (r[0] - l[0]);
}

}  // namespace frjf
