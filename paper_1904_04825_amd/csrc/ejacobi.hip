// Element-Jacobi preconditioner (Section 4.5): the diagonal element blocks
// P_e = shift I - dR_e/dq_e of the linear system, assembled by one-sided
// finite differences, inverted per element, and applied as z = P_e^{-1} r.
//
// Assembly.  Moving one state entry (v, k) of element e changes only the
// transformed fluxes at point k, the element's traces on the two xi-faces of
// k's eta-row and the two eta-faces of k's xi-column, and therefore the
// residual only along that row and column.  The kernel forms the finite
// difference of exactly those terms (flux at k, four common fluxes with the
// neighbours' traces held fixed), which equals [R_e(q + d e_j) - R_e(q)]
// up to rounding without re-evaluating the whole element.
// Inversion.  The raw blocks are written out and inverted in place with the
// block in MFMA registers and rank-16 updates on the matrix cores (gj_mfma.hip):
// FP64, or FP32 (the FP64 block rounded).  FP64 blocks of order 100 do not fit one
// wavefront's registers and keep the block rows in registers (gj_rows.hip).
// Application.  One 64-lane group per block row set: z_i = sum_j Pinv(i,j) r_j
// with the inverse stored column-major, so each step of the j loop is a
// coalesced load of one column.
#include <algorithm>
#include <type_traits>
#include <cmath>

#include "arnoldi.h"
#include "internal.h"
#include "physics.h"

namespace frjf {

template <int P>
struct EJ {
  static constexpr int n = P + 1, Np = n * n, Nb = 4 * Np;
  static constexpr int NT = ((Nb + 63) / 64) * 64;
  static constexpr int NZ = 4 * (2 * n - 1);  // structural nonzeros of a column
  static constexpr int LZ = NZ + 1;            // padded LDS leading dimension
};

struct AsmArgs {
  const double* U;
  const double* nodes;
  int nx, ny, nel;
  double gam, shift;
  void* out;
};

template <int P, int FLUX, typename T>
__global__ void __launch_bounds__(EJ<P>::NT) k_ejacobi_assemble(const AsmArgs a, const Basis B) {
  using C = EJ<P>;
  constexpr int n = C::n, Np = C::Np, Nb = C::Nb, NT = C::NT, LZ = C::LZ;
  // the block's structural nonzeros, per column: variable v, then the points of the
  // column point's eta-row (a = 0..n-1) and of its xi-column (b != its own b)
  __shared__ T Z[Nb * LZ];
  __shared__ double sq[4][Np], sF[4][Np], sG[4][Np], sIJ[Np];
  __shared__ double sqo[4][4][n], sqn[4][4][n], sFn[4][4][n];  // [face][var][j]
  __shared__ double sS[4][2];
  __shared__ double sMet[Np][4];  // xxi, xeta, yxi, yeta
  const int tid = threadIdx.x;
  const int el = blockIdx.x;
  const int ex = el % a.nx, ey = el / a.nx;
  const size_t nel = (size_t)a.nel;

  // base state, fluxes and metrics at the solution points
  for (int k = tid; k < Np; k += NT) {
    double q[4], c[8], f[4], g[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) q[v] = a.U[((size_t)v * nel + el) * Np + k];
    load_corners(a.nodes, a.nx, ex, ey, c);
    const Metric m = bilinear_metric(c, B.x[k % n], B.x[k / n]);
    euler_fluxes(q, a.gam, f, g);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sq[v][k] = q[v];
      sF[v][k] = m.yeta * f[v] - m.xeta * g[v];
      sG[v][k] = -m.yxi * f[v] + m.xxi * g[v];
    }
    sIJ[k] = 1.0 / m.J;
    sMet[k][0] = m.xxi;
    sMet[k][1] = m.xeta;
    sMet[k][2] = m.yxi;
    sMet[k][3] = m.yeta;
  }
  if (tid < 4) {
    double Sx, Sy;
    if (tid == 0) xi_face_normal(a.nodes, a.nx, ex, ey, &Sx, &Sy);
    else if (tid == 1) xi_face_normal(a.nodes, a.nx, (ex + 1 == a.nx) ? 0 : ex + 1, ey, &Sx, &Sy);
    else if (tid == 2) eta_face_normal(a.nodes, a.nx, ex, ey, &Sx, &Sy);
    else eta_face_normal(a.nodes, a.nx, ex, (ey + 1 == a.ny) ? 0 : ey + 1, &Sx, &Sy);
    sS[tid][0] = Sx;
    sS[tid][1] = Sy;
  }
  __syncthreads();
  // traces and base common fluxes on the four faces
  for (int t = tid; t < 4 * n; t += NT) {
    const int f = t / n, j = t % n;
    const bool xi_face = f < 2;
    const double* lw = (f == 0 || f == 2) ? B.lm : B.lp;
    const double* lo = (f == 0 || f == 2) ? B.lp : B.lm;
    int nex = ex, ney = ey;
    if (f == 0) nex = (ex == 0) ? a.nx - 1 : ex - 1;
    if (f == 1) nex = (ex + 1 == a.nx) ? 0 : ex + 1;
    if (f == 2) ney = (ey == 0) ? a.ny - 1 : ey - 1;
    if (f == 3) ney = (ey + 1 == a.ny) ? 0 : ey + 1;
    const size_t ne = (size_t)ney * a.nx + nex;
    double qo[4] = {0, 0, 0, 0}, qn[4] = {0, 0, 0, 0};
    for (int c = 0; c < n; ++c) {
      const int kk = xi_face ? j * n + c : c * n + j;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        qo[v] = fma(lw[c], sq[v][kk], qo[v]);
        qn[v] = fma(lo[c], a.U[((size_t)v * nel + ne) * Np + kk], qn[v]);
      }
    }
    double Fn[4];
    if (f == 0 || f == 2)
      common_flux<FLUX>(qn, qo, sS[f][0], sS[f][1], a.gam, Fn);
    else
      common_flux<FLUX>(qo, qn, sS[f][0], sS[f][1], a.gam, Fn);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sqo[f][v][j] = qo[v];
      sqn[f][v][j] = qn[v];
      sFn[f][v][j] = Fn[v];
    }
  }
  __syncthreads();

  // one finite-difference column per thread
  for (int jc = tid; jc < Nb; jc += NT) {
    const int vv = jc / Np, k = jc % Np, ak = k % n, bk = k / n;
    T* col = Z + jc * LZ;
    double q[4], f[4], g[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) q[v] = sq[v][k];
    const double delta = 1e-8 * fmax(1.0, fabs(q[vv]));
    q[vv] += delta;
    euler_fluxes(q, a.gam, f, g);
    double dF[4], dG[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      dF[v] = (sMet[k][3] * f[v] - sMet[k][1] * g[v]) - sF[v][k];
      dG[v] = (-sMet[k][2] * f[v] + sMet[k][0] * g[v]) - sG[v][k];
    }
    // change of (common flux - own flux trace) on the faces W, E (face point bk) and S, N (face point ak)
    double dJW[4], dJE[4], dJS[4], dJN[4];
    {
      double qL[4], qR[4], Fn[4];
      // W face: neighbour (left) fixed, own trace moved
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        qL[v] = sqn[0][v][bk];
        qR[v] = sqo[0][v][bk] + (v == vv ? B.lm[ak] * delta : 0.0);
      }
      common_flux<FLUX>(qL, qR, sS[0][0], sS[0][1], a.gam, Fn);
#pragma unroll
      for (int v = 0; v < 4; ++v) dJW[v] = (Fn[v] - sFn[0][v][bk]) - B.lm[ak] * dF[v];
      // E face: own (left) moved, neighbour fixed
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        qL[v] = sqo[1][v][bk] + (v == vv ? B.lp[ak] * delta : 0.0);
        qR[v] = sqn[1][v][bk];
      }
      common_flux<FLUX>(qL, qR, sS[1][0], sS[1][1], a.gam, Fn);
#pragma unroll
      for (int v = 0; v < 4; ++v) dJE[v] = (Fn[v] - sFn[1][v][bk]) - B.lp[ak] * dF[v];
      // S face at face point ak
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        qL[v] = sqn[2][v][ak];
        qR[v] = sqo[2][v][ak] + (v == vv ? B.lm[bk] * delta : 0.0);
      }
      common_flux<FLUX>(qL, qR, sS[2][0], sS[2][1], a.gam, Fn);
#pragma unroll
      for (int v = 0; v < 4; ++v) dJS[v] = (Fn[v] - sFn[2][v][ak]) - B.lm[bk] * dG[v];
      // N face
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        qL[v] = sqo[3][v][ak] + (v == vv ? B.lp[bk] * delta : 0.0);
        qR[v] = sqn[3][v][ak];
      }
      common_flux<FLUX>(qL, qR, sS[3][0], sS[3][1], a.gam, Fn);
#pragma unroll
      for (int v = 0; v < 4; ++v) dJN[v] = (Fn[v] - sFn[3][v][ak]) - B.lp[bk] * dG[v];
    }
    const double s = -1.0 / delta;  // column of -dR/dq: -(dR)/delta, with dR = -invJ * (...)
    // points of k's eta-row (a, bk): D[a][ak] dF + dJW gL[a] + dJE gR[a]
    for (int ia = 0; ia < n; ++ia) {
      const int kk = bk * n + ia;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double t = B.D[ia][ak] * dF[v] + dJW[v] * B.gL[ia] + dJE[v] * B.gR[ia];
        if (ia == ak) t += B.D[bk][bk] * dG[v] + dJS[v] * B.gL[bk] + dJN[v] * B.gR[bk];
        const T e = (T)(s * (-sIJ[kk] * t));
        col[v * (2 * n - 1) + ia] = (ia == ak && v == vv) ? (T)((double)e + a.shift) : e;
      }
    }
    // points of k's xi-column (ak, b), b != bk
    for (int ib = 0; ib < n; ++ib) {
      if (ib == bk) continue;
      const int kk = ib * n + ak;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double t = B.D[ib][bk] * dG[v] + dJS[v] * B.gL[ib] + dJN[v] * B.gR[ib];
        col[v * (2 * n - 1) + n + (ib < bk ? ib : ib - 1)] = (T)(s * (-sIJ[kk] * t));
      }
    }
  }
  __syncthreads();
  // write-out, column-major: thread = block row, so each store is contiguous across
  // the lanes; entries off the row point's eta-row and xi-column are zero
  T* out = reinterpret_cast<T*>(a.out) + (size_t)el * Nb * Nb;
  if (tid < Nb) {
    const int vr = tid / Np, kr = tid % Np, ar = kr % n, br = kr / n;
    const T* zr = Z + vr * (2 * n - 1);
#pragma unroll
    for (int col = 0; col < Nb; ++col) {
      const int kc = col % Np, ac = kc % n, bc = kc / n;
      T val = (T)0;
      if (br == bc)
        val = zr[col * LZ + ar];
      else if (ar == ac)
        val = zr[col * LZ + n + (br < bc ? br : br - 1)];
      out[(size_t)col * Nb + tid] = val;
    }
  }
}

// FP64 blocks rounded to FP32 (caller-provided blocks of the FP32 store).
__global__ void k_round_f32(const double* __restrict__ src, float* __restrict__ dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

// z = Pinv r per element (+ per-workgroup partial sums of ||z||^2), r optionally
// scaled by 1/(*r_scale) on load and stored back to r_store (fused normalisation of
// the Arnoldi vector).  The inverse is column-major, so column j of a block is
// Nb contiguous entries: a thread owns RPT consecutive rows and reads them with one
// load per column, a batch of columns in flight (the first batch issued before r is staged).  RPT = 1: one row per thread, the most
// threads; RPT = 16 / sizeof(T): 16-byte loads and dense lanes for large P = 4 stores.  EPB elements share a 256-thread
// workgroup; workgroups stride over groups of EPB elements.
template <int P, typename T, int RPT_>
struct SolveCfg {
  static constexpr int Np = (P + 1) * (P + 1), Nb = 4 * Np;
  static constexpr int RPT = RPT_;     // rows per thread
  static constexpr int TPE = Nb / RPT;  // threads per element
  static constexpr int EPB = 256 / TPE;  // elements per workgroup
  // columns in flight per thread: single rows (latency-bound stores that stay in the
  // last-level cache) 32 columns, FP32 ones at five waves per SIMD (the kernel's launch
  // bounds); 16-byte rows (large stores streamed from HBM) 8 columns, which measured
  // faster there
  static constexpr int JU0 = RPT == 1 ? 32 : 8;
  static constexpr int JU = JU0 < Nb ? JU0 : Nb;
  static_assert(Nb % RPT == 0, "whole rows per thread");
};

template <typename T, int RPT>
struct RowVec {
  typedef T type __attribute__((ext_vector_type(RPT)));
};
template <typename T>
struct RowVec<T, 1> {
  typedef T type;
};

template <typename V>
__device__ __forceinline__ double row_of(const V& a, int q) {
  if constexpr (sizeof(V) == sizeof(double) || sizeof(V) == sizeof(float))
    return (double)a;
  else
    return (double)a[q];
}

template <int P, typename T, int RPT>
__global__ void __launch_bounds__(256, (sizeof(T) == 4 && RPT == 1) ? 5 : 1) k_ejacobi_solve(const T* __restrict__ inv, const double* __restrict__ r,
                                                        const GivensIn gv, double* r_store, double* __restrict__ z,
                                                        int nel, double* partials, const int* skip) {
  using C = SolveCfg<P, T, RPT>;
  using V = typename RowVec<T, RPT>::type;
  constexpr int Np = C::Np, Nb = C::Nb, TPE = C::TPE, EPB = C::EPB;
  constexpr int JU = C::JU;  // columns in flight
  if (skip != nullptr && *skip) return;
  __shared__ T sr[EPB][Nb];
  const int tid = threadIdx.x;
  const int blk = tid / TPE, i = tid - blk * TPE;  // element of the group, row block
  // with gv: every workgroup forms ||r||^2 from the same partials in the same order,
  // workgroup 0 also finishes the Arnoldi step that produced r (CGS2: its Givens
  // update; DCGS2: stores ||r|| as the first-pass h_{j+1,j}, and rotates the
  // first-pass column on breakdown or NaN)
  const int ngroups = (nel + EPB - 1) / EPB;
  // single rows: the first JU columns of the first group are on their way during the
  // set-up below and while r goes through LDS (16-byte rows load after staging: held
  // through it they cost occupancy, measured slower)
  constexpr bool kEarly = C::RPT == 1;
  V m[JU];
  if constexpr (kEarly) {
    const int el = blockIdx.x * EPB + blk;
    if (blockIdx.x < ngroups && blk < EPB && el < nel) {
      const V* col = reinterpret_cast<const V*>(inv + (size_t)el * Nb * Nb) + i;
#pragma unroll
      for (int u = 0; u < JU; ++u) m[u] = col[(size_t)u * TPE];
    }
  }
  const bool scaled = gv.st != nullptr;
  double sc = 1.0;
  if (scaled) {
    __shared__ GivensLds GL;
    const double hn2 = block_sum_partials(gv.norm_part, gv.nb, GL.red);
    sc = 1.0 / sqrt(hn2);
    if (blockIdx.x == 0) {
      if (gv.lagged) {
        const double hn = sqrt(hn2), w0 = gv.st->w0;
        if (tid == 0) gv.st->hn = hn;
        if (!(hn > 1e-14 * w0)) givens_first_pass(gv.st, hn, gv.M, GL);  // breakdown or NaN
      } else {
        givens_step(gv.st, hn2, gv.M, GL);
      }
    }
  }
  double zz = 0.0;
  for (int grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int el = grp * EPB + blk;
    const bool live = blk < EPB && el < nel;
    const V* col = reinterpret_cast<const V*>(inv + (size_t)(live ? el : 0) * Nb * Nb) + i;  // rows RPT i .. RPT i + RPT - 1
    if (kEarly && live && grp != (int)blockIdx.x) {
#pragma unroll
      for (int u = 0; u < JU; ++u) m[u] = col[(size_t)u * TPE];
    }
    __syncthreads();
    for (int t = tid; t < EPB * Nb; t += 256) {
      const int e = t / Nb, jj = t - e * Nb, el = grp * EPB + e;
      if (el >= nel) continue;
      const int v = jj / Np, k = jj - v * Np;
      const size_t gi = ((size_t)v * nel + el) * Np + k;
      double rv = r[gi];
      if (scaled) {
        rv *= sc;
        if (r_store != nullptr) r_store[gi] = rv;
      }
      sr[e][jj] = (T)rv;
    }
    __syncthreads();
    if (live) {
      V acc0 = {}, acc1 = {};
      int j = 0;
      for (; j + JU <= Nb; j += JU) {
        if (j > 0 || !kEarly) {
#pragma unroll
          for (int u = 0; u < JU; ++u) m[u] = col[(size_t)(j + u) * TPE];
        }
#pragma unroll
        for (int u = 0; u + 1 < JU; u += 2) {
          acc0 += m[u] * sr[blk][j + u];
          acc1 += m[u + 1] * sr[blk][j + u + 1];
        }
        if constexpr (JU % 2 == 1) acc0 += m[JU - 1] * sr[blk][j + JU - 1];
      }
      for (; j < Nb; ++j) acc0 += col[(size_t)j * TPE] * sr[blk][j];
      const V acc = acc0 + acc1;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int row = RPT * i + q;
        const double zi = row_of(acc, q);
        const int v = row / Np, k = row - v * Np;
        z[((size_t)v * nel + el) * Np + k] = zi;
        zz = fma(zi, zi, zz);
      }
    }
  }
  if (partials == nullptr) return;
  __shared__ double red[4];
  zz = wave_sum(zz);
  if ((tid & 63) == 0) red[tid >> 6] = zz;
  __syncthreads();
  if (tid == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ---------------------------------------------------------------- LU-SGS passes
// The matrix-free LU-SGS preconditioner (Section 4.5 names it beside element-Jacobi):
// symmetric block Gauss-Seidel over the two checkerboard colours c = (ex + ey) mod 2,
// with the element blocks D as its diagonal and the couplings between colours applied
// matrix-free through Jacobian-free products (the host driver, lusgs_apply):
//   PASS 1, colour 0: out = D^{-1} r, out = 0 on colour 1 (with gv, r is first scaled by
//           1/||r|| and stored to r_store on every element, as in k_ejacobi_solve);
//   PASS 2, colour 1: t = D^{-1}(r - w): out = t and out2 = t there, out2 = 0 on colour 0
//           (out left as it is on colour 0);
//   PASS 3, colour 0: out = y - D^{-1} w, out = y on colour 1.
// Per-workgroup partial sums of ||out||^2 (PASS 2: of ||out2||^2).  Workgroups take
// groups of EPB elements of the active colour (element a of colour c: row a / (nx/2),
// column 2 (a mod nx/2) + ((c + row) mod 2)), then stride over the other colour's entries.
struct LusgsArgs {
  const double* r;   // PASS 1, 2
  const double* w;   // PASS 2, 3
  const double* y;   // PASS 3
  double* out;
  double* out2;      // PASS 2
  double* r_store;   // PASS 1 with gv
  int nx, nel;
};

template <int P, typename T, int PASS>
__global__ void __launch_bounds__(256) k_lusgs_pass(const T* __restrict__ inv, const LusgsArgs a, const GivensIn gv,
                                                    double* partials, const int* skip) {
  using C = SolveCfg<P, T, 1>;
  constexpr int Np = C::Np, Nb = C::Nb, TPE = C::TPE, EPB = C::EPB, JU = C::JU;
  constexpr int act = (PASS == 2) ? 1 : 0;  // active colour
  if (skip != nullptr && *skip) return;
  __shared__ T sr[EPB][Nb];
  const int tid = threadIdx.x;
  const int blk = tid / TPE, i = tid - blk * TPE;
  const int hx = a.nx >> 1, nact = a.nel >> 1;
  const size_t nel = (size_t)a.nel;
  const bool scaled = PASS == 1 && gv.st != nullptr;
  double sc = 1.0;
  if (scaled) {
    __shared__ GivensLds GL;
    const double hn2 = block_sum_partials(gv.norm_part, gv.nb, GL.red);
    sc = 1.0 / sqrt(hn2);
    if (blockIdx.x == 0) {
      if (gv.lagged) {
        const double hn = sqrt(hn2), w0 = gv.st->w0;
        if (tid == 0) gv.st->hn = hn;
        if (!(hn > 1e-14 * w0)) givens_first_pass(gv.st, hn, gv.M, GL);
      } else {
        givens_step(gv.st, hn2, gv.M, GL);
      }
    }
  }
  auto element = [&](int ai, int colour) {
    const int ey = ai / hx, ex = 2 * (ai - ey * hx) + ((colour + ey) & 1);
    return ey * a.nx + ex;
  };
  double acc2 = 0.0;
  const int ngroups = (nact + EPB - 1) / EPB;
  for (int grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int ai = grp * EPB + blk;
    const bool live = blk < EPB && ai < nact;
    const int el = live ? element(ai, act) : 0;
    __syncthreads();
    for (int t = tid; t < EPB * Nb; t += 256) {
      const int e = t / Nb, jj = t - e * Nb, ae = grp * EPB + e;
      if (ae >= nact) continue;
      const int ee = element(ae, act);
      const int v = jj / Np, k = jj - v * Np;
      const size_t gi = ((size_t)v * nel + ee) * Np + k;
      double rv;
      if constexpr (PASS == 1) {
        rv = a.r[gi];
        if (scaled) {
          rv *= sc;
          if (a.r_store != nullptr) a.r_store[gi] = rv;
        }
      } else if constexpr (PASS == 2) {
        rv = a.r[gi] - a.w[gi];
      } else {
        rv = a.w[gi];
      }
      sr[e][jj] = (T)rv;
    }
    __syncthreads();
    if (live) {
      const T* col = inv + (size_t)el * Nb * Nb + i;
      double acc0 = 0.0, acc1 = 0.0;
      T m[JU];
      int j = 0;
      for (; j + JU <= Nb; j += JU) {
#pragma unroll
        for (int u = 0; u < JU; ++u) m[u] = col[(size_t)(j + u) * TPE];
#pragma unroll
        for (int u = 0; u + 1 < JU; u += 2) {
          acc0 += (double)(m[u] * sr[blk][j + u]);
          acc1 += (double)(m[u + 1] * sr[blk][j + u + 1]);
        }
        if constexpr (JU % 2 == 1) acc0 += (double)(m[JU - 1] * sr[blk][j + JU - 1]);
      }
      for (; j < Nb; ++j) acc0 += (double)(col[(size_t)j * TPE] * sr[blk][j]);
      const double zi = acc0 + acc1;
      const int v = i / Np, k = i - v * Np;
      const size_t gi = ((size_t)v * nel + el) * Np + k;
      double o;
      if constexpr (PASS == 3) {
        o = a.y[gi] - zi;
      } else {
        o = zi;
      }
      a.out[gi] = o;
      if constexpr (PASS == 2) a.out2[gi] = o;
      acc2 = fma(o, o, acc2);
    }
  }
  // the other colour's entries
  const size_t nother = (size_t)4 * nact * Np;
  for (size_t t = (size_t)blockIdx.x * 256 + tid; t < nother; t += (size_t)gridDim.x * 256) {
    const int v = (int)(t / ((size_t)nact * Np));
    const size_t rem = t - (size_t)v * nact * Np;
    const int ai = (int)(rem / Np), k = (int)(rem - (size_t)ai * Np);
    const size_t gi = ((size_t)v * nel + element(ai, 1 - act)) * Np + k;
    if constexpr (PASS == 1) {
      a.out[gi] = 0.0;
      if (scaled && a.r_store != nullptr) a.r_store[gi] = a.r[gi] * sc;
    } else if constexpr (PASS == 2) {
      a.out2[gi] = 0.0;
    } else {
      const double yv = a.y[gi];
      a.out[gi] = yv;
      acc2 = fma(yv, yv, acc2);
    }
  }
  if (partials == nullptr) return;
  __shared__ double red[4];
  acc2 = wave_sum(acc2);
  if ((tid & 63) == 0) red[tid >> 6] = acc2;
  __syncthreads();
  if (tid == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

template <int P, typename T>
static hipError_t lusgs_pt(const fr_disc* d, const T* f, int pass, const LusgsArgs& a, const GivensIn& gv,
                           double* partials, const int* skip, int* nb_out, hipStream_t s) {
  constexpr int EPB = SolveCfg<P, T, 1>::EPB;
  const int ngroups = (d->nel / 2 + EPB - 1) / EPB;
  const int nb = std::max(1, std::min(ngroups, kRedBlocks));
  *nb_out = nb;
  if (pass == 1)
    hipLaunchKernelGGL((k_lusgs_pass<P, T, 1>), dim3(nb), dim3(256), 0, s, f, a, gv, partials, skip);
  else if (pass == 2)
    hipLaunchKernelGGL((k_lusgs_pass<P, T, 2>), dim3(nb), dim3(256), 0, s, f, a, gv, partials, skip);
  else
    hipLaunchKernelGGL((k_lusgs_pass<P, T, 3>), dim3(nb), dim3(256), 0, s, f, a, gv, partials, skip);
  return hipGetLastError();
}

template <int P>
static hipError_t lusgs_p(const fr_disc* d, const void* f, int precision, int pass, const LusgsArgs& a,
                          const GivensIn* gvp, double* partials, const int* skip, int* nb_out, hipStream_t s) {
  const GivensIn gv = gvp != nullptr ? *gvp : GivensIn{nullptr, nullptr, 0, 0, 0};
  if (gv.st != nullptr && (gv.nb < 1 || gv.nb > kRedBlocks || gv.norm_part == nullptr)) return hipErrorInvalidValue;
  if (precision == FR_F32)
    return lusgs_pt<P, float>(d, (const float*)f, pass, a, gv, partials, skip, nb_out, s);
  return lusgs_pt<P, double>(d, (const double*)f, pass, a, gv, partials, skip, nb_out, s);
}

hipError_t launch_lusgs_pass(const fr_disc* d, const void* factors, int precision, int pass, const double* r,
                             const double* w, const double* y, double* out, double* out2, const GivensIn* gv,
                             double* r_store, double* partials, int* nparts, const int* skip, hipStream_t s) {
  if ((d->nx & 1) || (d->ny & 1) || pass < 1 || pass > 3) return hipErrorInvalidValue;
  const LusgsArgs a{r, w, y, out, out2, r_store, d->nx, d->nel};
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (d->p) {
    case 2: e = lusgs_p<2>(d, factors, precision, pass, a, gv, partials, skip, &nb, s); break;
    case 3: e = lusgs_p<3>(d, factors, precision, pass, a, gv, partials, skip, &nb, s); break;
    case 4: e = lusgs_p<4>(d, factors, precision, pass, a, gv, partials, skip, &nb, s); break;
    case 5: e = lusgs_p<5>(d, factors, precision, pass, a, gv, partials, skip, &nb, s); break;
    case 6: e = lusgs_p<6>(d, factors, precision, pass, a, gv, partials, skip, &nb, s); break;
  }
  if (nparts != nullptr) *nparts = nb;
  return e;
}

template <int P, int FLUX>
static hipError_t asm_pf(const fr_disc* d, const AsmArgs& a, int precision, int invert, hipStream_t s) {
  dim3 grid(d->nel), block(EJ<P>::NT);
  if (precision == FR_F32) {
    // FP32: the FP64 blocks rounded on the way out, then inverted in place on MFMA
    if (!invert) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_ejacobi_assemble<P, FLUX, float>), grid, block, 0, s, a, d->basis);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_invert_f32(EJ<P>::Nb, static_cast<float*>(a.out), d->nel, s);
  } else {
    // FP64: the raw blocks, then their inverses in place
    hipLaunchKernelGGL((k_ejacobi_assemble<P, FLUX, double>), grid, block, 0, s, a, d->basis);
    if (invert) {
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      return launch_invert_f64(EJ<P>::Nb, static_cast<double*>(a.out), d->nel, s);
    }
  }
  return hipGetLastError();
}

template <int P>
static hipError_t asm_p(const fr_disc* d, const AsmArgs& a, int precision, int invert, hipStream_t s) {
  return d->flux == FR_ROE ? asm_pf<P, 1>(d, a, precision, invert, s) : asm_pf<P, 0>(d, a, precision, invert, s);
}

hipError_t launch_ns_ejacobi_assemble(const fr_disc* d, const double* U, double shift, void* out, int precision,
                                      int invert, double* grad, hipStream_t s);

hipError_t launch_ejacobi_assemble(const fr_disc* d, const double* U, double shift, void* out, int precision,
                                   int invert, double* grad, hipStream_t s) {
  if (d->physics == FR_NS_BR1) return launch_ns_ejacobi_assemble(d, U, shift, out, precision, invert, grad, s);
  const AsmArgs a{U, d->nodes, d->nx, d->ny, d->nel, d->phys.gamma, shift, out};
  switch (d->p) {
    case 2: return asm_p<2>(d, a, precision, invert, s);
    case 3: return asm_p<3>(d, a, precision, invert, s);
    case 4: return asm_p<4>(d, a, precision, invert, s);
    case 5: return asm_p<5>(d, a, precision, invert, s);
    case 6: return asm_p<6>(d, a, precision, invert, s);
  }
  return hipErrorInvalidValue;
}

template <int P>
static hipError_t inv_p(const fr_disc* d, const double* blocks, void* out, int precision, hipStream_t s) {
  constexpr int Nb = EJ<P>::Nb;
  if (precision == FR_F32) {
    const size_t total = (size_t)d->nel * Nb * Nb;
    hipLaunchKernelGGL(k_round_f32, dim3((unsigned)std::min<size_t>((total + 255) / 256, 65536)), dim3(256), 0, s,
                       blocks, static_cast<float*>(out), total);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_invert_f32(Nb, static_cast<float*>(out), d->nel, s);
  }
  const hipError_t e = hipMemcpyAsync(out, blocks, (size_t)d->nel * Nb * Nb * sizeof(double),
                                      hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  return launch_invert_f64(Nb, static_cast<double*>(out), d->nel, s);
}

hipError_t launch_ejacobi_invert_blocks(const fr_disc* d, const double* blocks, void* out, int precision,
                                        hipStream_t s) {
  switch (d->p) {
    case 2: return inv_p<2>(d, blocks, out, precision, s);
    case 3: return inv_p<3>(d, blocks, out, precision, s);
    case 4: return inv_p<4>(d, blocks, out, precision, s);
    case 5: return inv_p<5>(d, blocks, out, precision, s);
    case 6: return inv_p<6>(d, blocks, out, precision, s);
  }
  return hipErrorInvalidValue;
}

// 16-byte rows where one row per thread leaves lanes idle (Nb = 100: two blocks per
// 256-thread workgroup use 200 lanes) and the store does not stay in the 256 MB
// last-level cache.
constexpr size_t kWideSolveBytes = size_t(256) << 20;

template <int P, typename T, int RPT>
static hipError_t solve_ptr(const fr_disc* d, const void* f, const double* r, const GivensIn& gv, double* r_store,
                            double* z, double* partials, const int* skip, int* nb_out, hipStream_t s) {
  constexpr int EPB = SolveCfg<P, T, RPT>::EPB;
  const int ngroups = (d->nel + EPB - 1) / EPB;
  const int nb = std::min(ngroups, kRedBlocks);
  *nb_out = nb;
  hipLaunchKernelGGL((k_ejacobi_solve<P, T, RPT>), dim3(nb), dim3(256), 0, s, (const T*)f, r, gv, r_store, z,
                     d->nel, partials, skip);
  return hipGetLastError();
}

template <int P>
static hipError_t solve_p(const fr_disc* d, const void* f, int precision, const double* r, const GivensIn* gvp,
                          double* r_store, double* z, double* partials, int* nparts, double* nrm2, const int* skip,
                          hipStream_t s) {
  constexpr int Nb = 4 * (P + 1) * (P + 1);
  const GivensIn gv = gvp != nullptr ? *gvp : GivensIn{nullptr, nullptr, 0, 0, 0};
  if (gv.st != nullptr && (gv.nb < 1 || gv.nb > kRedBlocks || gv.norm_part == nullptr)) return hipErrorInvalidValue;
  double* part = (nrm2 != nullptr || nparts != nullptr) ? partials : nullptr;
  const size_t store = (size_t)d->nel * Nb * Nb * (precision == FR_F32 ? sizeof(float) : sizeof(double));
  const bool wide = P == 4 && store >= kWideSolveBytes;
  int nb = 0;
  hipError_t e;
  if (precision == FR_F32)
    e = wide ? solve_ptr<P, float, 4>(d, f, r, gv, r_store, z, part, skip, &nb, s)
             : solve_ptr<P, float, 1>(d, f, r, gv, r_store, z, part, skip, &nb, s);
  else
    e = wide ? solve_ptr<P, double, 2>(d, f, r, gv, r_store, z, part, skip, &nb, s)
             : solve_ptr<P, double, 1>(d, f, r, gv, r_store, z, part, skip, &nb, s);
  if (nparts != nullptr) *nparts = nb;
  if (e != hipSuccess || nrm2 == nullptr) return e;
  return launch_finalize(partials, nb, 1, 1, nrm2, skip, s);
}

hipError_t launch_ejacobi_solve(const fr_disc* d, const void* factors, int precision, const double* r,
                                const GivensIn* gv, double* r_store, double* z, double* partials,
                                int* nparts, double* nrm2, const int* skip, hipStream_t s) {
  switch (d->p) {
    case 2: return solve_p<2>(d, factors, precision, r, gv, r_store, z, partials, nparts, nrm2, skip, s);
    case 3: return solve_p<3>(d, factors, precision, r, gv, r_store, z, partials, nparts, nrm2, skip, s);
    case 4: return solve_p<4>(d, factors, precision, r, gv, r_store, z, partials, nparts, nrm2, skip, s);
    case 5: return solve_p<5>(d, factors, precision, r, gv, r_store, z, partials, nparts, nrm2, skip, s);
    case 6: return solve_p<6>(d, factors, precision, r, gv, r_store, z, partials, nparts, nrm2, skip, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace frjf
