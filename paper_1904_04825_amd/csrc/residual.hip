// FR/CPR residual of the 2D Euler equations (Section 3) and the fused
// Jacobian-free product (Section 4.5), one kernel template:
//   MODE 0: out = R(U)
//   MODE 1: out = shift v - [R(U + e v) - R0] / e
//   MODE 2: out = b - (shift v - [R(U + e v) - R0] / e)      (GMRES true residual)
//
// A workgroup owns a TX x TY tile of elements and gives one thread to every
// element line.  The operators are tensor products of 1D ones, so the work
// splits into line passes whose basis coefficients are compile-time indexed
// (scalar registers) and whose derivatives stay in vector registers:
//   halo   the solution traces of the elements around the tile on the faces
//          they share with it, straight from global memory;
//   rows   thread (e, j) takes row j (constant eta) of element e: the state
//          goes to LDS, F = y_eta f - x_eta g, D_xi F, and the W/E traces of
//          q and of F;
//   cols   the same thread takes column j (constant xi) from LDS:
//          G = -y_xi f + x_xi g, D_eta G, and the S/N traces of q and of G;
//   faces  one common flux |S| f^com per face point of the tile, the state
//          on the -xi / -eta side first; a face on the tile border is also
//          computed by the neighbouring tile from bit-identical traces, so
//          both sides see the same flux and the scheme stays conservative;
//   out    jumps F^num - F^l times the Radau correction derivatives, the
//          column results handed to the row threads through LDS, R = -div/J.
#include <algorithm>

#include "internal.h"
#include "physics.h"
#include "wavesum.h"

namespace frjf {

// Tiles: a large one for big meshes, a small one so that small meshes still
// spread over every compute unit.
template <int P, bool BIG>
struct LineTile;
#ifndef FRJF_TILE_P2
#define FRJF_TILE_P2 16, 5, 7, 3
#endif
#ifndef FRJF_TILE_P3
#define FRJF_TILE_P3 8, 8, 4, 4
#endif
#ifndef FRJF_TILE_P4
#define FRJF_TILE_P4 10, 5, 5, 2
#endif
template <bool BIG, int TXB, int TYB, int TXS, int TYS>
struct TilePick {
  static constexpr int TX = BIG ? TXB : TXS, TY = BIG ? TYB : TYS;
};
template <bool BIG> struct LineTile<2, BIG> : TilePick<BIG, FRJF_TILE_P2> {};
template <bool BIG> struct LineTile<3, BIG> : TilePick<BIG, FRJF_TILE_P3> {};
template <bool BIG> struct LineTile<4, BIG> : TilePick<BIG, FRJF_TILE_P4> {};
#ifndef FRJF_TILE_P5
#define FRJF_TILE_P5 7, 3, 3, 3
#endif
#ifndef FRJF_TILE_P6
#define FRJF_TILE_P6 6, 3, 3, 3
#endif
template <bool BIG> struct LineTile<5, BIG> : TilePick<BIG, FRJF_TILE_P5> {};
template <bool BIG> struct LineTile<6, BIG> : TilePick<BIG, FRJF_TILE_P6> {};

#ifndef FRJF_SPLIT_SMALL
#define FRJF_SPLIT_SMALL 1
#endif
template <int P, bool BIG>
struct LineCfg {
  static constexpr int n = P + 1, Np = n * n;
  // element stride of the LDS state: row writes and column reads without bank conflicts
  static constexpr int ES = (n == 4) ? Np + 3 : Np;
  static constexpr int TX = LineTile<P, BIG>::TX, TY = LineTile<P, BIG>::TY, NE = TX * TY;
  static constexpr int NL = NE * n;                 // element lines
  // small tiles: one set of wavefronts takes the rows (xi), another the columns (eta) of
  // every element, so the two passes and their faces run side by side
  static constexpr bool SPLIT = FRJF_SPLIT_SMALL && !BIG;
  static constexpr int NTH = (NL + 63) / 64 * 64;   // threads of one role
  static constexpr int NT = SPLIT ? 2 * NTH : NTH;
  static constexpr int NFX = TY * (TX + 1) * n;     // xi-face points
  static constexpr int NFE = (TY + 1) * TX * n;     // eta-face points
  static constexpr int NF = NFX + NFE;
  static constexpr int NH = 2 * (TX + TY) * n;      // halo lines
  // trace slots: W, E, S, N faces of the tile's elements, then the halo's W, E, S, N sides
  static constexpr int SW = 0, SE = NE * n, SS = 2 * NE * n, SN = 3 * NE * n;
  static constexpr int SHW = 4 * NE * n, SHE = SHW + TY * n, SHS = SHE + TY * n, SHN = SHS + TX * n;
  static constexpr int NS = SHN + TX * n;
  static constexpr int QS = NE * ES;                // variable stride of the LDS state
  static constexpr int A = (4 * QS > 4 * NF) ? 4 * QS : 4 * NF;
};

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

// arr[t] for a per-thread t < n, by selects over compile-time indexed entries
template <int n>
__device__ __forceinline__ double pick(const double (&arr)[kMaxN], int t) {
  double r = arr[0];
#pragma unroll
  for (int c = 1; c < n; ++c) r = (t == c) ? arr[c] : r;
  return r;
}

// 1/a to full double precision: hardware estimate and two Newton steps
__device__ __forceinline__ double rcp64(double a) {
  double r = __builtin_amdgcn_rcp(a);
  double e = fma(-a, r, 1.0);
  r = fma(r, e, r);
  e = fma(-a, r, 1.0);
  return fma(r, e, r);
}

// sqrt(a) for positive normal a: hardware 1/sqrt(a) estimate refined by
// Goldschmidt's coupled iteration for sqrt(a) and 1/(2 sqrt(a)).
__device__ __forceinline__ double sqrt64(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  double g = a * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, a);
  g = fma(d, h, g);
  d = fma(-g, g, a);
  return fma(d, h, g);
}

// Rusanov flux with the area-weighted normal S: |S| f^com =
// (f_S(qL) + f_S(qR))/2 - Lambda (qR - qL)/2, f_S = f S_x + g S_y,
// Lambda = max over both sides of |u.S| + c|S|.
__device__ __forceinline__ void rusanov_face(const double qL[4], const double qR[4], double Sx, double Sy,
                                             double gam, double out[4]) {
  const double magS = sqrt64(Sx * Sx + Sy * Sy);
  double lam = 0.0;
  double fs[2][4];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const double* q = side ? qR : qL;
    const double ir = rcp64(q[0]);
    const double u = q[1] * ir, v = q[2] * ir;
    const double p = (gam - 1.0) * (q[3] - 0.5 * (q[1] * u + q[2] * v));
    const double uS = u * Sx + v * Sy;
    fs[side][0] = q[0] * uS;
    fs[side][1] = q[1] * uS + p * Sx;
    fs[side][2] = q[2] * uS + p * Sy;
    fs[side][3] = (q[3] + p) * uS;
    lam = fmax(lam, fabs(uS) + sqrt64(gam * p * ir) * magS);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) out[v] = 0.5 * (fs[0][v] + fs[1][v]) - 0.5 * lam * (qR[v] - qL[v]);
}

template <int FLUX>
__device__ __forceinline__ void face_flux(const double qL[4], const double qR[4], double Sx, double Sy,
                                          double gam, double out[4]) {
  if constexpr (FLUX == 0)
    rusanov_face(qL, qR, Sx, Sy, gam, out);
  else
    roe_flux(qL, qR, Sx, Sy, gam, out);
}

// f and g of q = (rho, rho u, rho v, E) combined into a transformed flux
// alpha f + beta g.
__device__ __forceinline__ void transformed_flux(const double q[4], double gam, double alpha, double beta,
                                                 double out[4]) {
  const double ir = rcp64(q[0]);
  const double u = q[1] * ir, v = q[2] * ir;
  const double p = (gam - 1.0) * (q[3] - 0.5 * (q[1] * u + q[2] * v));
  const double un = alpha * u + beta * v;  // contravariant velocity
  out[0] = q[0] * un;
  out[1] = fma(q[1], un, alpha * p);
  out[2] = fma(q[2], un, beta * p);
  out[3] = (q[3] + p) * un;
}

// Tile of the linear sequence number k: first element column / row and the
// live element counts (the last tile row / column may be ragged).
template <int TX, int TY>
struct TileIdx {
  int ex0, ey0, mX, mY;
  __device__ __forceinline__ TileIdx(int k, int T, int ntx, int nx, int ny) {
    const int tile = xcd_remap(k, T);
    ex0 = (tile % ntx) * TX;
    ey0 = (tile / ntx) * TY;
    mX = min(TX, nx - ex0);
    mY = min(TY, ny - ey0);
  }
};

template <int P, int FLUX, int MODE, bool BIG, int DOTS = 0>
__global__ void __launch_bounds__((LineCfg<P, BIG>::NT)) k_euler(const ResArgs a, const MeshArgs g, const Basis B) {
  static_assert(DOTS == 0 || (MODE == 1 && !BIG), "the first DCGS2 pass rides on small-tile JF products only");
  using C = LineCfg<P, BIG>;
  constexpr int n = C::n, Np = C::Np, ES = C::ES, TX = C::TX, TY = C::TY, NT = C::NT;
  constexpr int QS = C::QS, NS = C::NS, NF = C::NF;
  constexpr int RUN = TX * Np, NIT = (TY * RUN + NT - 1) / NT, NHI = (C::NH + NT - 1) / NT;
  __shared__ double sA[C::A];        // state, then common face fluxes, then column results
  __shared__ double sT[4 * C::NS];   // solution traces

  if (MODE != 0 && a.skip != nullptr && *a.skip) return;
  const int tid = threadIdx.x;
  const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + TY - 1) / TY;
  const TileIdx<TX, TY> ti(blockIdx.x, ntx * nty, ntx, g.nx, g.ny);
  const int ex0 = ti.ex0, ey0 = ti.ey0, mX = ti.mX, mY = ti.mY;
  const size_t nel = (size_t)g.nel, vstride = nel * Np;
  double e = 0.0, ie = 0.0;
  bool zero_v = false;
  // e = eps / rms(v): on small meshes every wavefront adds the partial sums of ||v||^2
  // itself, after the tile's and the halo's loads are on their way (the halo keeps U and
  // v apart until e is known); on large meshes ||v||^2 is one finished value
  constexpr bool kLateE = MODE != 0 && !BIG && P <= 3;  // P4: the separate halo registers cost occupancy
  auto eps_of = [&]() {
    if (a.eps_mode == FR_EPS_RMS) {
      const double n2 = (!BIG && a.nrm2_part != nullptr) ? wave_sum_partials(a.nrm2_part, a.nrm2_nb) : *a.nrm2;
      if (n2 > 0.0)
        e = a.eps / sqrt(n2 / (double)(4 * nel * Np));
      else
        zero_v = true;
    } else {
      e = a.eps;
    }
    ie = zero_v ? 0.0 : 1.0 / e;
  };
  if constexpr (MODE != 0 && !kLateE) eps_of();

  // ---- the tile's state and the halo lines.  Every global load of the phase is
  // issued before the first use, so the tile and halo reads overlap.  Each tile row
  // of a variable is one contiguous run of mX * Np doubles, read with consecutive
  // lanes; U (and v) are combined when the state is written to LDS.
  double pu[NIT][4], pv[MODE ? NIT : 1][4];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int idx = tid + it * NT, ry = idx / RUN, kk = idx - ry * RUN;
    if (idx < TY * RUN && ry < mY && kk < mX * Np) {
      const size_t base = ((size_t)(ey0 + ry) * g.nx + ex0) * Np + kk;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        pu[it][v] = a.U[v * vstride + base];
        if constexpr (MODE != 0) pv[MODE ? it : 0][v] = a.V[v * vstride + base];
      }
    }
  }
  {
    // ---- halo lines: the row (west / east neighbour) or column (south / north
    // neighbour) of the element across a border face, loaded before the state lands
    double hq[NHI][n][4];
    double hv[kLateE ? NHI : 1][kLateE ? n : 1][4];
    int hslot[NHI];
    bool hplus[NHI];
#pragma unroll
    for (int it = 0; it < NHI; ++it) {
      const int h = tid + it * NT;
      hslot[it] = -1;
      hplus[it] = false;
      size_t base = 0;
      int stride = 1;
      if (h < 2 * TY * n) {  // rows of the west / east neighbours
        const int side = h / (TY * n), r = h - side * (TY * n), ly = r / n, j = r - ly * n;
        if (ly < mY) {
          int hx = side ? ex0 + mX : ex0 - 1;
          hx = hx < 0 ? hx + g.nx : (hx >= g.nx ? hx - g.nx : hx);
          base = ((size_t)(ey0 + ly) * g.nx + hx) * Np + j * n;
          hslot[it] = (side ? C::SHE : C::SHW) + ly * n + j;
          hplus[it] = side == 0;  // the west neighbour's east face, the east neighbour's west face
        }
      } else if (h < C::NH) {  // columns of the south / north neighbours
        const int h2 = h - 2 * TY * n;
        const int side = h2 / (TX * n), r = h2 - side * (TX * n), lx = r / n, i = r - lx * n;
        if (lx < mX) {
          int hy = side ? ey0 + mY : ey0 - 1;
          hy = hy < 0 ? hy + g.ny : (hy >= g.ny ? hy - g.ny : hy);
          base = ((size_t)hy * g.nx + ex0 + lx) * Np + i;
          stride = n;
          hslot[it] = (side ? C::SHN : C::SHS) + lx * n + i;
          hplus[it] = side == 0;  // the south neighbour's north face
        }
      }
      if (hslot[it] >= 0) {
#pragma unroll
        for (int c = 0; c < n; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const size_t gi = v * vstride + base + c * stride;
            if constexpr (kLateE) {
              hq[it][c][v] = a.U[gi];
              hv[kLateE ? it : 0][kLateE ? c : 0][v] = a.V[gi];
            } else {
              hq[it][c][v] = state_at<MODE>(a, gi, e);
            }
          }
      }
    }
    if constexpr (kLateE) {
      eps_of();
#pragma unroll
      for (int it = 0; it < NHI; ++it)
#pragma unroll
        for (int c = 0; c < n; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v) hq[it][c][v] = fma(e, hv[kLateE ? it : 0][kLateE ? c : 0][v], hq[it][c][v]);
    }

    // ---- the state into LDS
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = tid + it * NT, ry = idx / RUN, kk = idx - ry * RUN;
      if (idx < TY * RUN && ry < mY && kk < mX * Np) {
        const int dst = (ry * TX + kk / Np) * ES + kk % Np;
#pragma unroll
        for (int v = 0; v < 4; ++v) sA[v * QS + dst] = MODE ? fma(e, pv[MODE ? it : 0][v], pu[it][v]) : pu[it][v];
      }
    }
#pragma unroll
    for (int it = 0; it < NHI; ++it) {
      if (hslot[it] < 0) continue;
      double tr[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int c = 0; c < n; ++c) {
        const double w = hplus[it] ? B.lp[c] : B.lm[c];
#pragma unroll
        for (int v = 0; v < 4; ++v) tr[v] = fma(w, hq[it][c][v], tr[v]);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) sT[v * NS + hslot[it]] = tr[v];
    }
    __syncthreads();

    // ---- rows (with split roles, the first C::NTH threads; the others take the columns)
    const bool colrole = C::SPLIT && tid >= C::NTH;
    const int lt = colrole ? tid - C::NTH : tid;
    const int le = lt / n, t = lt - le * n;
    const int lx = le % TX, ly = le / TX;
    const bool live = lt < C::NL && lx < mX && ly < mY;
    const bool rows = live && !colrole, cols = live && (colrole || !C::SPLIT);
    const double tp = pick<n>(B.x, t);  // eta of row t, xi of column t
    // bilinear map: x_xi = ax + bx eta, x_eta = cx + dx xi (and the same for y)
    double ax = 0, bx = 0, ay = 0, by = 0, cx = 0, dx = 0, cy = 0, dy = 0;
    double nW[2] = {0, 0}, nS[2] = {0, 0};  // normals of the west and south faces
    double dF[n][4], FlW[4], FlE[4];
    if (live) {
      double c[8];
      load_corners(g.nodes, g.nx, ex0 + lx, ey0 + ly, c);
      ax = 0.25 * ((c[2] - c[0]) + (c[6] - c[4]));
      bx = 0.25 * ((c[6] - c[4]) - (c[2] - c[0]));
      ay = 0.25 * ((c[3] - c[1]) + (c[7] - c[5]));
      by = 0.25 * ((c[7] - c[5]) - (c[3] - c[1]));
      cx = 0.25 * ((c[4] - c[0]) + (c[6] - c[2]));
      dx = 0.25 * ((c[6] - c[2]) - (c[4] - c[0]));
      cy = 0.25 * ((c[5] - c[1]) + (c[7] - c[3]));
      dy = 0.25 * ((c[7] - c[3]) - (c[5] - c[1]));
      // xi-faces S = (y_eta, -x_eta), eta-faces S = (-y_xi, x_xi), from the edge's end nodes;
      // the node pair of an edge is the same for both tiles sharing it
      nW[0] = 0.5 * (c[5] - c[1]);
      nW[1] = -0.5 * (c[4] - c[0]);
      nS[0] = -0.5 * (c[3] - c[1]);
      nS[1] = 0.5 * (c[2] - c[0]);
    }
    if (rows) {
      double q[n][4];
#pragma unroll
      for (int cc = 0; cc < n; ++cc)
#pragma unroll
        for (int v = 0; v < 4; ++v) q[cc][v] = sA[v * QS + le * ES + t * n + cc];
      double qW[4] = {0, 0, 0, 0}, qE[4] = {0, 0, 0, 0};
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        FlW[v] = 0.0;
        FlE[v] = 0.0;
#pragma unroll
        for (int i = 0; i < n; ++i) dF[i][v] = 0.0;
      }
#pragma unroll
      for (int cc = 0; cc < n; ++cc) {
        const double xeta = fma(dx, B.x[cc], cx), yeta = fma(dy, B.x[cc], cy);
        double F[4];
        transformed_flux(q[cc], g.gam, yeta, -xeta, F);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
#pragma unroll
          for (int i = 0; i < n; ++i) dF[i][v] = fma(B.D[i][cc], F[v], dF[i][v]);
          qW[v] = fma(B.lm[cc], q[cc][v], qW[v]);
          qE[v] = fma(B.lp[cc], q[cc][v], qE[v]);
          FlW[v] = fma(B.lm[cc], F[v], FlW[v]);
          FlE[v] = fma(B.lp[cc], F[v], FlE[v]);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        sT[v * NS + C::SW + le * n + t] = qW[v];
        sT[v * NS + C::SE + le * n + t] = qE[v];
      }
    }
    if constexpr (!C::SPLIT) __syncthreads();

    // ---- columns
    double dG[n][4], GlS[4], GlN[4];
    if (cols) {
      const double xeta = fma(dx, tp, cx), yeta = fma(dy, tp, cy);
      double qS[4] = {0, 0, 0, 0}, qN[4] = {0, 0, 0, 0};
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        GlS[v] = 0.0;
        GlN[v] = 0.0;
#pragma unroll
        for (int j = 0; j < n; ++j) dG[j][v] = 0.0;
      }
#pragma unroll
      for (int r = 0; r < n; ++r) {
        double q[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) q[v] = sA[v * QS + le * ES + r * n + t];
        const double xxi = fma(bx, B.x[r], ax), yxi = fma(by, B.x[r], ay);
        double G[4];
        transformed_flux(q, g.gam, -yxi, xxi, G);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
#pragma unroll
          for (int j = 0; j < n; ++j) dG[j][v] = fma(B.D[j][r], G[v], dG[j][v]);
          qS[v] = fma(B.lm[r], q[v], qS[v]);
          qN[v] = fma(B.lp[r], q[v], qN[v]);
          GlS[v] = fma(B.lm[r], G[v], GlS[v]);
          GlN[v] = fma(B.lp[r], G[v], GlN[v]);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        sT[v * NS + C::SS + le * n + t] = qS[v];
        sT[v * NS + C::SN + le * n + t] = qN[v];
      }
    }
    __syncthreads();

    // ---- faces: one common flux per face point, the state on the -xi / -eta side first.
    // Slots: xi-face point j of face f in tile row fy at (fy (TX+1) + f) n + j, then
    // eta-face point i of face row fy, column fx at NFX + (fy TX + fx) n + i.
    const int nstride = g.nx + 1;
    if (rows) {  // the west face point t of the thread's element
      double qL[4], qR[4], Fn[4];
      const int sL = (lx == 0) ? C::SHW + ly * n + t : C::SE + (le - 1) * n + t;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        qL[v] = sT[v * NS + sL];
        qR[v] = sT[v * NS + C::SW + le * n + t];
      }
      face_flux<FLUX>(qL, qR, nW[0], nW[1], g.gam, Fn);
      const int fW = (ly * (TX + 1) + lx) * n + t;
#pragma unroll
      for (int v = 0; v < 4; ++v) sA[v * NF + fW] = Fn[v];
    }
    if (cols) {  // the south face point t
      double qL[4], qR[4], Fn[4];
      const int sL = (ly == 0) ? C::SHS + lx * n + t : C::SN + (le - TX) * n + t;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        qL[v] = sT[v * NS + sL];
        qR[v] = sT[v * NS + C::SS + le * n + t];
      }
      face_flux<FLUX>(qL, qR, nS[0], nS[1], g.gam, Fn);
      const int fS = C::NFX + (ly * TX + lx) * n + t;
#pragma unroll
      for (int v = 0; v < 4; ++v) sA[v * NF + fS] = Fn[v];
    }
    for (int b = tid; b < (TY + TX) * n; b += NT) {  // the tile's east and north border faces
      int sL, sR, slot;
      double Sx, Sy;
      if (b < TY * n) {
        const int fy = b / n, j = b - fy * n;
        if (fy >= mY) continue;
        int ix = ex0 + mX;
        if (ix >= g.nx) ix -= g.nx;
        const double* pA = g.nodes + 2 * ((ey0 + fy) * nstride + ix);
        const double* pB = pA + 2 * nstride;
        Sx = 0.5 * (pB[1] - pA[1]);
        Sy = -0.5 * (pB[0] - pA[0]);
        sL = C::SE + (fy * TX + mX - 1) * n + j;
        sR = C::SHE + fy * n + j;
        slot = (fy * (TX + 1) + mX) * n + j;
      } else {
        const int b2 = b - TY * n, fx = b2 / n, i = b2 - fx * n;
        if (fx >= mX) continue;
        int iy = ey0 + mY;
        if (iy >= g.ny) iy -= g.ny;
        const double* pA = g.nodes + 2 * (iy * nstride + ex0 + fx);
        Sx = -0.5 * (pA[3] - pA[1]);
        Sy = 0.5 * (pA[2] - pA[0]);
        sL = C::SN + ((mY - 1) * TX + fx) * n + i;
        sR = C::SHN + fx * n + i;
        slot = C::NFX + (mY * TX + fx) * n + i;
      }
      double qL[4], qR[4], Fn[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        qL[v] = sT[v * NS + sL];
        qR[v] = sT[v * NS + sR];
      }
      face_flux<FLUX>(qL, qR, Sx, Sy, g.gam, Fn);
#pragma unroll
      for (int v = 0; v < 4; ++v) sA[v * NF + slot] = Fn[v];
    }
    __syncthreads();

    // ---- corrections: rows take the W/E jumps, columns the S/N jumps
    if (rows) {
      const int fW = (ly * (TX + 1) + lx) * n + t;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double jW = sA[v * NF + fW] - FlW[v], jE = sA[v * NF + fW + n] - FlE[v];
#pragma unroll
        for (int i = 0; i < n; ++i) dF[i][v] = fma(B.gL[i], jW, fma(B.gR[i], jE, dF[i][v]));
      }
    }
    if (cols) {
      const int fS = C::NFX + (ly * TX + lx) * n + t;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double jS = sA[v * NF + fS] - GlS[v], jN = sA[v * NF + fS + TX * n] - GlN[v];
#pragma unroll
        for (int i = 0; i < n; ++i) dG[i][v] = fma(B.gL[i], jS, fma(B.gR[i], jN, dG[i][v]));
      }
    }
    // v and R0 of the write-out positions, on their way during the last passes
    double ov[MODE ? NIT : 1][4], orr[MODE ? NIT : 1][4];
    if constexpr (MODE != 0) {
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        const int idx = tid + it * NT, ry = idx / RUN, kk = idx - ry * RUN;
        if (idx < TY * RUN && ry < mY && kk < mX * Np) {
          const size_t base = ((size_t)(ey0 + ry) * g.nx + ex0) * Np + kk;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            ov[MODE ? it : 0][v] = a.V[v * vstride + base];
            orr[MODE ? it : 0][v] = a.R0[v * vstride + base];
          }
        }
      }
    }
    __syncthreads();
    if (cols) {
#pragma unroll
      for (int r = 0; r < n; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) sA[v * QS + le * ES + r * n + t] = dG[r][v];
    }
    __syncthreads();

    // ---- R = -(D_xi F + D_eta G + corrections) / J on row t, back into LDS
    if (rows) {
      const double xxi = fma(bx, tp, ax), yxi = fma(by, tp, ay);
#pragma unroll
      for (int i = 0; i < n; ++i) {
        const double xeta = fma(dx, B.x[i], cx), yeta = fma(dy, B.x[i], cy);
        const double iJ = rcp64(xxi * yeta - xeta * yxi);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double* o = &sA[v * QS + le * ES + t * n + i];
          *o = -(dF[i][v] + *o) * iJ;
        }
      }
    }
    __syncthreads();

    // ---- coalesced write-out, the matrix-free combinations on the fly (with DOTS, the
    // first DCGS2 pass over w = A v: the basis vectors' entries at the written positions
    // and their sums, as k_dcgs_dots forms them)
    constexpr int NA = 2 * DOTS;
    double dacc[DOTS > 0 ? NA : 1];
    double oacc = 0.0;  // mode 2: ||b - A x||^2 of the written entries
#pragma unroll
    for (int q = 0; q < (DOTS > 0 ? NA : 1); ++q) dacc[q] = 0.0;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = tid + it * NT, ry = idx / RUN, kk = idx - ry * RUN;
      if (idx < TY * RUN && ry < mY && kk < mX * Np) {
        const size_t base = ((size_t)(ey0 + ry) * g.nx + ex0) * Np + kk;
        const int src = (ry * TX + kk / Np) * ES + kk % Np;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const size_t gi = v * vstride + base;
          const double R = sA[v * QS + src];
          if constexpr (MODE == 0) {
            a.out[gi] = R;
          } else {
            const double av = zero_v ? 0.0 : a.shift * ov[MODE ? it : 0][v] - (R - orr[MODE ? it : 0][v]) * ie;
            if constexpr (MODE == 1) {
              a.out[gi] = av;
            } else {
              const double o = a.B[gi] - av;
              a.out[gi] = o;
              oacc = fma(o, o, oacc);
            }
            if constexpr (DOTS > 0) {
              const size_t ndof = 4 * vstride;
              double vr[DOTS > 0 ? DOTS : 1];
#pragma unroll
              for (int q = 0; q < DOTS; ++q) vr[q] = a.dV[(size_t)min(q, a.dnv - 1) * ndof + gi];
              const double vj = a.dV[(size_t)(a.dnv - 1) * ndof + gi];
#pragma unroll
              for (int q = 0; q < DOTS; ++q) dacc[q] = fma(vr[q], av, dacc[q]);
#pragma unroll
              for (int q = 0; q + 1 < DOTS; ++q) dacc[DOTS + q] = fma(vr[q], vj, dacc[DOTS + q]);
              dacc[NA - 1] = fma(av, av, dacc[NA - 1]);
            }
          }
        }
      }
    }
    if constexpr (MODE == 2 && !BIG) {
      if (a.opart != nullptr) {
        __shared__ double ored[NT / 64];
        oacc = wave_sum(oacc);
        if ((tid & 63) == 0) ored[tid >> 6] = oacc;
        __syncthreads();
        if (tid == 0) {
          double r = 0.0;
#pragma unroll
          for (int q = 0; q < NT / 64; ++q) r += ored[q];
          a.opart[blockIdx.x] = r;
        }
      }
    }
    if constexpr (DOTS > 0) {
      __shared__ double dred[NT / 64][NA > 0 ? NA : 1];
      int off;
      if (wave_multi_sum<NA>(dacc, off)) {
#pragma unroll
        for (int q = 0; q < multi_sum_count(NA); ++q) dred[tid >> 6][off + q] = dacc[q];
      }
      __syncthreads();
      if (tid < NA) {
        double r = 0.0;
#pragma unroll
        for (int q = 0; q < NT / 64; ++q) r += dred[q][tid];
        a.dpart[(size_t)tid * kRedBlocks + blockIdx.x] = r;
      }
    }
  }
}

// Large tiles once the mesh gives every compute unit several of them.
#ifndef FRJF_BIG_TILE_MIN_BLOCKS
#define FRJF_BIG_TILE_MIN_BLOCKS 2048
#endif
constexpr int kBigTileMinBlocks = FRJF_BIG_TILE_MIN_BLOCKS;

template <int P, int FLUX, bool BIG>
static hipError_t launch_euler_tile(const fr_disc* d, int mode, const ResArgs& a, hipStream_t s) {
  using C = LineCfg<P, BIG>;
  const int ntx = (d->nx + C::TX - 1) / C::TX, nty = (d->ny + C::TY - 1) / C::TY;
  const MeshArgs g{d->nodes, d->nx, d->ny, d->nel, d->phys.gamma};
  dim3 grid(ntx * nty), block(C::NT);
  if constexpr (BIG) {
    if (a.opart != nullptr) return hipErrorInvalidValue;
  } else {
    if (a.opart != nullptr && (mode != 2 || ntx * nty > kRedBlocks)) return hipErrorInvalidValue;
  }
  if (a.dV != nullptr) {
    // the JF product with the first DCGS2 pass: small tiles, one partial row slot per tile
    if constexpr (BIG) {
      return hipErrorInvalidValue;
    } else {
      if (mode != 1 || a.dnv < 1 || a.dnv > kJfDotsMax || a.dpart == nullptr || ntx * nty > kRedBlocks)
        return hipErrorInvalidValue;
      if (a.dnv <= 4)
        hipLaunchKernelGGL((k_euler<P, FLUX, 1, false, 4>), grid, block, 0, s, a, g, d->basis);
      else if (a.dnv <= 8)
        hipLaunchKernelGGL((k_euler<P, FLUX, 1, false, 8>), grid, block, 0, s, a, g, d->basis);
      else if (a.dnv <= 12)
        hipLaunchKernelGGL((k_euler<P, FLUX, 1, false, 12>), grid, block, 0, s, a, g, d->basis);
      else if (a.dnv <= 16)
        hipLaunchKernelGGL((k_euler<P, FLUX, 1, false, 16>), grid, block, 0, s, a, g, d->basis);
      else
        hipLaunchKernelGGL((k_euler<P, FLUX, 1, false, 20>), grid, block, 0, s, a, g, d->basis);
      return hipGetLastError();
    }
  }
  if (mode == 0)
    hipLaunchKernelGGL((k_euler<P, FLUX, 0, BIG>), grid, block, 0, s, a, g, d->basis);
  else if (mode == 1)
    hipLaunchKernelGGL((k_euler<P, FLUX, 1, BIG>), grid, block, 0, s, a, g, d->basis);
  else
    hipLaunchKernelGGL((k_euler<P, FLUX, 2, BIG>), grid, block, 0, s, a, g, d->basis);
  return hipGetLastError();
}

// ||v||^2 from its partial sums for kernels that do not add them themselves
static hipError_t finish_nrm2(int mode, ResArgs& a, hipStream_t s) {
  if (mode == 0 || a.nrm2_part == nullptr || a.eps_mode != FR_EPS_RMS) return hipSuccess;
  const hipError_t e = launch_finalize(a.nrm2_part, a.nrm2_nb, 1, 1, a.nrm2, a.skip, s);
  a.nrm2_part = nullptr;
  return e;
}

template <int P>
static long big_tiles(const fr_disc* d) {
  using C = LineCfg<P, true>;
  return (long)((d->nx + C::TX - 1) / C::TX) * ((d->ny + C::TY - 1) / C::TY);
}

template <int P>
static int small_tiles(const fr_disc* d) {
  using C = LineCfg<P, false>;
  return ((d->nx + C::TX - 1) / C::TX) * ((d->ny + C::TY - 1) / C::TY);
}

template <int P>
static int dots_blocks_p(const fr_disc* d) {
  if (big_tiles<P>(d) >= kBigTileMinBlocks) return 0;
  const int nb = small_tiles<P>(d);
  return nb <= kRedBlocks ? nb : 0;
}

int residual_dots_blocks(const fr_disc* d) {
  if (d->physics != FR_EULER) return 0;
  switch (d->p) {
    case 2: return dots_blocks_p<2>(d);
    case 3: return dots_blocks_p<3>(d);
    case 4: return dots_blocks_p<4>(d);
    case 5: return dots_blocks_p<5>(d);
    case 6: return dots_blocks_p<6>(d);
  }
  return 0;
}

template <int P, int FLUX>
static hipError_t launch_euler_pf(const fr_disc* d, int mode, const ResArgs& a, hipStream_t s) {
  if (big_tiles<P>(d) < kBigTileMinBlocks) return launch_euler_tile<P, FLUX, false>(d, mode, a, s);
  // many tiles: one finalize kernel instead of every wavefront reading the partials
  ResArgs b = a;
  const hipError_t e = finish_nrm2(mode, b, s);
  if (e != hipSuccess) return e;
  return launch_euler_tile<P, FLUX, true>(d, mode, b, s);
}

template <int P>
static hipError_t launch_euler_p(const fr_disc* d, int mode, const ResArgs& a, hipStream_t s) {
  return d->flux == FR_ROE ? launch_euler_pf<P, 1>(d, mode, a, s) : launch_euler_pf<P, 0>(d, mode, a, s);
}

hipError_t launch_ns_residual(const fr_disc* d, int mode, const ResArgs& a, hipStream_t s);

hipError_t launch_residual(const fr_disc* d, int mode, const ResArgs& a, hipStream_t s) {
  if (d->physics == FR_NS_BR1) {
    ResArgs b = a;
    const hipError_t e = finish_nrm2(mode, b, s);
    if (e != hipSuccess) return e;
    return launch_ns_residual(d, mode, b, s);
  }
  switch (d->p) {
    case 2: return launch_euler_p<2>(d, mode, a, s);
    case 3: return launch_euler_p<3>(d, mode, a, s);
    case 4: return launch_euler_p<4>(d, mode, a, s);
    case 5: return launch_euler_p<5>(d, mode, a, s);
    case 6: return launch_euler_p<6>(d, mode, a, s);
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
                            double* partials, double* out, hipStream_t s) {
  const MeshArgs g{d->nodes, d->nx, d->ny, d->nel, d->phys.gamma};
  VortexPrm P;
  for (int i = 0; i < 14; ++i) P.v[i] = prm[i];
  hipLaunchKernelGGL(k_l2_vortex, dim3(256), dim3(256), 0, s, g, d->basis, U, var, t, P, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(partials, 256, 2, 2, out, nullptr, s);
}

}  // namespace frjf
