// Host drivers of the implicit solver (Section 4): restarted flexible GMRES
// with the Jacobian-free product and the element-Jacobi preconditioner, the
// ROW, ESDIRK and BDF2 time steps, and pseudo-transient continuation (PTC)
// with SER pseudo-time stepping and rejection.  Every vector operation runs
// on the device; the host only sequences kernels and reads scalar norms.
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"
#include "solvers.h"

namespace frjf {

// ---------------------------------------------------------------- coefficient tables
// ROW schemes in the transformed form of eq. Rosenbrock_General.
// ROW2: 3-stage, order 2, stiffly accurate, L-stable, gamma = 1/4 (standard form:
//   beta_21 = 1/2, b = (5/8, 1/8, 1/4), alpha_21 = alpha_31 = alpha_32 = 1/2),
//   used because the ROS2PR coefficients are not available.
// ROW3: ROS34PW2 (Rang & Angermann 2005), converted from the published standard form.
// ROW4: RODASP (Steinebach 1995), transformed form as published.
namespace {

void to_transformed(int s, const double* alpha, const double* gam, const double* b, RowScheme* out) {
  // Gamma lower triangular: invert by forward substitution, then
  // A = alpha Gamma^{-1}, C = diag(1/gamma) - Gamma^{-1}, m = b Gamma^{-1}.
  double Gi[36] = {0};
  for (int c = 0; c < s; ++c) {
    for (int r = 0; r < s; ++r) {
      double v = (r == c) ? 1.0 : 0.0;
      for (int k = 0; k < r; ++k) v -= gam[r * s + k] * Gi[k * s + c];
      Gi[r * s + c] = v / gam[r * s + r];
    }
  }
  out->s = s;
  out->gamma = gam[0];
  for (int r = 0; r < s; ++r)
    for (int c = 0; c < s; ++c) {
      double a = 0.0;
      for (int k = 0; k < s; ++k) a += alpha[r * s + k] * Gi[k * s + c];
      out->a[r][c] = (c < r) ? a : 0.0;
      out->c[r][c] = (c < r) ? -Gi[r * s + c] : 0.0;
    }
  for (int c = 0; c < s; ++c) {
    double m = 0.0;
    for (int k = 0; k < s; ++k) m += b[k] * Gi[k * s + c];
    out->m[c] = m;
  }
}

RowScheme make_row2() {
  const double g = 0.25;
  const double alpha[9] = {0, 0, 0, 0.5, 0, 0, 0.5, 0.5, 0};
  const double b[3] = {5.0 / 8.0, 1.0 / 8.0, 0.25};
  // Gamma = beta - alpha with beta_21 = 1/2 and the last row of beta equal to b
  const double gam[9] = {g, 0, 0, 0.5 - 0.5, g, 0, b[0] - 0.5, b[1] - 0.5, g};
  RowScheme r{};
  to_transformed(3, alpha, gam, b, &r);
  return r;
}

RowScheme make_ros34pw2() {
  const double g = 0.4358665215084590;
  double alpha[16] = {0}, gam[16] = {0};
  alpha[1 * 4 + 0] = 0.87173304301691801;
  alpha[2 * 4 + 0] = 0.84457060015369423;
  alpha[2 * 4 + 1] = -0.11299064236484185;
  alpha[3 * 4 + 2] = 1.0;
  gam[1 * 4 + 0] = -0.87173304301691801;
  gam[2 * 4 + 0] = -0.90338057013044082;
  gam[2 * 4 + 1] = 0.054180672388095326;
  gam[3 * 4 + 0] = 0.24212380706095346;
  gam[3 * 4 + 1] = -1.2232505839045147;
  gam[3 * 4 + 2] = 0.54526025533510214;
  for (int i = 0; i < 4; ++i) gam[i * 4 + i] = g;
  const double b[4] = {0.24212380706095346, -1.2232505839045147, 1.5452602553351020, 0.43586652150845900};
  RowScheme r{};
  to_transformed(4, alpha, gam, b, &r);
  return r;
}

RowScheme make_rodasp() {
  RowScheme r{};
  r.s = 6;
  r.gamma = 0.25;
  const double A[6][5] = {{0, 0, 0, 0, 0},
                          {3.0, 0, 0, 0, 0},
                          {1.831036793486759, 0.4955183967433795, 0, 0, 0},
                          {2.304376582692669, -0.05249275245743001, -1.176798761832782, 0, 0},
                          {-7.170454962423024, -4.741636671481785, -16.31002631330971, -1.062004044111401, 0},
                          {-7.170454962423024, -4.741636671481785, -16.31002631330971, -1.062004044111401, 1.0}};
  const double C[6][5] = {{0, 0, 0, 0, 0},
                          {-12.0, 0, 0, 0, 0},
                          {-8.791795173947035, -2.207865586973518, 0, 0, 0},
                          {10.81793056857153, 6.780270611428266, 19.53485944642410, 0, 0},
                          {34.19095006749676, 15.49671153725963, 54.74760875964130, 14.16005392148534, 0},
                          {34.62605830930532, 15.30084976114473, 56.99955578662667, 18.40807009793095,
                           -5.714285714285717}};
  const double m[6] = {-7.170454962423024, -4.741636671481785, -16.31002631330971, -1.062004044111401, 1.0, 1.0};
  for (int i = 0; i < 6; ++i) {
    for (int j = 0; j < 5; ++j) {
      r.a[i][j] = A[i][j];
      r.c[i][j] = C[i][j];
    }
    r.m[i] = m[i];
  }
  return r;
}

// ESDIRK Butcher tables (eq. ESDIRK2 form: explicit first stage, a_ii = omega).
EsdirkScheme make_esdirk2() {
  EsdirkScheme e{};
  const double g = 1.0 - 1.0 / std::sqrt(2.0);
  e.s = 3;
  e.gamma = g;
  e.a[1][0] = g;
  e.a[1][1] = g;
  e.a[2][0] = 0.5 * (1.0 - g);
  e.a[2][1] = 0.5 * (1.0 - g);
  e.a[2][2] = g;
  for (int i = 0; i < 3; ++i) e.b[i] = e.a[2][i];
  return e;
}

// Kennedy & Carpenter ARK3(2)4L[2]SA, implicit part (the ESDIRK3 of Bijl et al. 2002).
EsdirkScheme make_esdirk3() {
  EsdirkScheme e{};
  const double g = 1767732205903.0 / 4055673282236.0;
  e.s = 4;
  e.gamma = g;
  e.a[1][0] = g;
  e.a[1][1] = g;
  e.a[2][0] = 2746238789719.0 / 10658868560708.0;
  e.a[2][1] = -640167445237.0 / 6845629431997.0;
  e.a[2][2] = g;
  e.a[3][0] = 1471266399579.0 / 7840856788654.0;
  e.a[3][1] = -4482444167858.0 / 7529755066697.0;
  e.a[3][2] = 11266239266428.0 / 11593286722821.0;
  e.a[3][3] = g;
  for (int i = 0; i < 4; ++i) e.b[i] = e.a[3][i];
  return e;
}

// Kennedy & Carpenter ARK4(3)6L[2]SA, implicit part (the ESDIRK4 of Bijl et al. 2002).
EsdirkScheme make_esdirk4() {
  EsdirkScheme e{};
  const double g = 0.25;
  e.s = 6;
  e.gamma = g;
  e.a[1][0] = g;
  e.a[1][1] = g;
  e.a[2][0] = 8611.0 / 62500.0;
  e.a[2][1] = -1743.0 / 31250.0;
  e.a[2][2] = g;
  e.a[3][0] = 5012029.0 / 34652500.0;
  e.a[3][1] = -654441.0 / 2922500.0;
  e.a[3][2] = 174375.0 / 388108.0;
  e.a[3][3] = g;
  e.a[4][0] = 15267082809.0 / 155376265600.0;
  e.a[4][1] = -71443401.0 / 120774400.0;
  e.a[4][2] = 730878875.0 / 902184768.0;
  e.a[4][3] = 2285395.0 / 8070912.0;
  e.a[4][4] = g;
  e.a[5][0] = 82889.0 / 524892.0;
  e.a[5][1] = 0.0;
  e.a[5][2] = 15625.0 / 83664.0;
  e.a[5][3] = 69875.0 / 102672.0;
  e.a[5][4] = -2260.0 / 8211.0;
  e.a[5][5] = g;
  for (int i = 0; i < 6; ++i) e.b[i] = e.a[5][i];
  return e;
}

}  // namespace

const RowScheme* row_scheme(int id) {
  static const RowScheme r2 = make_row2(), r3 = make_ros34pw2(), r4 = make_rodasp();
  switch (id) {
    case FR_ROW2: return &r2;
    case FR_ROW3: return &r3;
    case FR_ROW4: return &r4;
  }
  return nullptr;
}

const EsdirkScheme* esdirk_scheme(int id) {
  static const EsdirkScheme e2 = make_esdirk2(), e3 = make_esdirk3(), e4 = make_esdirk4();
  switch (id) {
    case FR_ESDIRK2: return &e2;
    case FR_ESDIRK3: return &e3;
    case FR_ESDIRK4: return &e4;
  }
  return nullptr;
}

// ---------------------------------------------------------------- workspace
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t ns_trace_bytes(const fr_disc* d) {
  // BR1: corrected-gradient traces on 4 faces x (P+1) points x 4 variables x 2 components
  return d->physics == FR_NS_BR1 ? (size_t)d->nel * 4 * d->n * 4 * 2 * sizeof(double) : 0;
}

// Partial sums: the grid-stride reductions and the two sets of CGS partial rows use
// at most kRedBlocks x (kMaxM + 2) slots, the preconditioner application one slot per
// workgroup (at most one per element).
size_t partials_count(const fr_disc* d) {
  return std::max<size_t>((size_t)kRedBlocks * (kMaxM + 2), (size_t)d->nel);
}

size_t gmres_bytes(const fr_disc* d, int m) {
  // V (m + 1), Z (m), w, r and the LU-SGS vectors (3)
  return align256(ns_trace_bytes(d)) + align256(sizeof(GmState)) + 256 +
         align256(sizeof(double) * partials_count(d)) + align256(sizeof(double) * d->ndof) * (size_t)(2 * m + 6);
}

size_t small_bytes(const fr_disc* d) { return 256 + align256(sizeof(double) * partials_count(d)); }

Carver::Carver(void* base) : p((char*)base) {}
void* Carver::take(size_t bytes) {
  void* r = p;
  p += align256(bytes);
  return r;
}

GmWork carve_gmres(Carver& c, const fr_disc* d, int m) {
  GmWork w{};
  w.grad = d->physics == FR_NS_BR1 ? (double*)c.take(ns_trace_bytes(d)) : nullptr;
  w.st = (GmState*)c.take(sizeof(GmState));
  w.scal = (double*)c.take(256);
  w.partials = (double*)c.take(sizeof(double) * partials_count(d));
  w.V = (double*)c.take(sizeof(double) * d->ndof * (size_t)(m + 1));
  w.Z = (double*)c.take(sizeof(double) * d->ndof * (size_t)m);
  w.w = (double*)c.take(sizeof(double) * d->ndof);
  w.r = (double*)c.take(sizeof(double) * d->ndof);
  for (int i = 0; i < 3; ++i) w.t[i] = (double*)c.take(sizeof(double) * d->ndof);
  return w;
}

// Read `bytes` from device into the pinned host scratch and wait.
static fr_status read_sync(const fr_disc* d, void* dst, const void* dev, size_t bytes, hipStream_t s) {
  char* slot = (char*)d->h_pinned + 1024;  // the first KiB holds the Arnoldi status slots
  FR_HIP(hipMemcpyAsync(slot, dev, bytes, hipMemcpyDeviceToHost, s));
  FR_HIP(hipStreamSynchronize(s));
  std::memcpy(dst, slot, bytes);
  return FR_OK;
}

fr_status device_norm(const fr_disc* d, const double* x, double* partials, double* dev_out,
                      double* host_out, hipStream_t s) {
  FR_HIP(launch_norm2(x, d->ndof, partials, dev_out, nullptr, s));
  double v = 0.0;
  fr_status st = read_sync(d, &v, dev_out, sizeof(double), s);
  if (st != FR_OK) return st;
  *host_out = std::sqrt(v);
  return FR_OK;
}

// ---------------------------------------------------------------- LU-SGS
fr_status lusgs_apply(const fr_disc* d, const void* factors, int prec, const ResArgs& ra, const double* r,
                      const GivensIn* gv, double* r_store, double* z, GmWork& W, double* zpart, int* np,
                      const int* skip, long* evals, hipStream_t s) {
  double* y = W.t[0];   // forward sweep: y_R, then y_B
  double* yb = W.t[1];  // y on black elements, zero on red
  double* w = W.t[2];   // Jacobian-free products
  double* part = W.partials + kPartZ;
  const double* rr = (gv != nullptr && r_store != nullptr) ? r_store : r;  // r / ||r|| once stored
  int nb = 0;
  // y_R = D_R^{-1} r_R (y_B = 0)
  FR_HIP(launch_lusgs_pass(d, factors, prec, 1, r, nullptr, nullptr, y, nullptr, gv, r_store, part, &nb, skip, s));
  ResArgs a = ra;
  a.V = y;
  a.out = w;
  a.nrm2_part = part;
  a.nrm2_nb = nb;
  a.skip = skip;
  a.dV = nullptr;
  a.opart = nullptr;
  FR_HIP(launch_residual(d, 1, a, s));  // w = A y: its black part is A_BR y_R
  // y_B = D_B^{-1}(r_B - A_BR y_R), also into yb (red part zero)
  FR_HIP(launch_lusgs_pass(d, factors, prec, 2, rr, w, nullptr, y, yb, nullptr, nullptr, part, &nb, skip, s));
  a.V = yb;
  a.nrm2_nb = nb;
  FR_HIP(launch_residual(d, 1, a, s));  // w = A yb: its red part is A_RB y_B
  // z_R = y_R - D_R^{-1} A_RB y_B, z_B = y_B
  FR_HIP(launch_lusgs_pass(d, factors, prec, 3, nullptr, w, y, z, nullptr, nullptr, nullptr, zpart, np, skip, s));
  if (evals != nullptr) *evals += 2;
  return FR_OK;
}

// ---------------------------------------------------------------- FGMRES
fr_status gmres_core(const fr_disc* d, const void* factors, int prec, const double* U, const double* R0,
                     double shift, const double* b, double* x, bool x_is_zero, const fr_gmres_opts& o,
                     fr_gmres_stats* stats, GmWork& W, hipStream_t s, bool plain_fallback, int* fell_back,
                     const fr_pmg* mg) {
  const size_t n = d->ndof;
  const int m = o.m;
  const int max_iters = o.max_iters > 0 ? o.max_iters : 50 * m;
  if (o.precond == FR_PC_LUSGS && (d->physics != FR_EULER || (d->nx & 1) || (d->ny & 1)))
    return set_error(FR_EINVAL, "LU-SGS preconditioner: Euler meshes with even nx and ny only");
  if (o.precond == FR_PC_PMG && !pmg_compatible(d, mg))
    return set_error(FR_EINVAL, "p-multigrid preconditioner: no matching coarse level (fr_pmg_factor)");
  fr_gmres_stats S{};
  double* nz = W.scal + 0;     // ||z||^2 or ||x||^2 for the JF epsilon
  double* beta2 = W.scal + 1;  // ||r||^2

  ResArgs ra{};
  ra.U = U;
  ra.R0 = R0;
  ra.eps = o.eps > 0 ? o.eps : 1e-8;
  ra.eps_mode = o.eps_mode;
  ra.shift = shift;
  ra.nrm2 = nz;
  ra.grad = W.grad;

  const double* rsrc = b;
  double bnorm = -1.0;  // ||b||, the residual of the zero (plain) guess
  if (fell_back != nullptr) *fell_back = 0;
  // a supplied guess that may fall back to zero needs ||b|| and ||r_0|| on the host;
  // otherwise the first cycle's start kernel takes the reference norm and the checks
  const bool host_start = !x_is_zero && plain_fallback;
  if (host_start) {
    double bb = 0.0;
    FR_HIP(launch_norm2(b, n, W.partials, beta2, nullptr, s));
    fr_status r0 = read_sync(d, &bb, beta2, sizeof(double), s);
    if (r0 != FR_OK) return r0;
    bnorm = std::sqrt(bb);
  }
  if (!x_is_zero) {
    FR_HIP(launch_norm2(x, n, W.partials, nz, nullptr, s));
    ResArgs a2 = ra;
    a2.V = x;
    a2.B = b;
    a2.out = W.r;
    FR_HIP(launch_residual(d, 2, a2, s));
    S.residual_evals++;
    rsrc = W.r;
  }
  FR_HIP(launch_norm2(rsrc, n, W.partials, beta2, nullptr, s));
  fr_status rs = FR_OK;
  double ref = o.ref_norm > 0 ? o.ref_norm : 0.0;  // 0: the start kernel takes ||r_0||
  if (host_start) {
    double b2 = 0.0;
    rs = read_sync(d, &b2, beta2, sizeof(double), s);
    if (rs != FR_OK) return rs;
    double beta = std::sqrt(b2);
    if (!(beta < bnorm)) {
      // the supplied guess is no better than zero: start from zero
      const double* none[1];
      double zc[1];
      FR_HIP(launch_lincomb(x, 0, none, zc, n, s));
      FR_HIP(launch_norm2(b, n, W.partials, beta2, nullptr, s));
      rsrc = b;
      beta = bnorm;
      if (fell_back != nullptr) *fell_back = 1;
    }
    S.r_ref = o.ref_norm > 0 ? o.ref_norm : bnorm;
    S.r_final = beta;
    if (!std::isfinite(beta)) {
      *stats = S;
      return FR_ENAN;
    }
    if (beta <= o.rtol * S.r_ref) {
      S.converged = 1;
      *stats = S;
      return FR_OK;
    }
    ref = S.r_ref;
  }
  // mapped host status written by the Givens kernel after every Arnoldi step
  // orthogonalisation: DCGS2 (two passes over V per step, the Hessenberg column final
  // one step later) up to m = 32, CGS2 beyond
  const bool dcgs = dcgs2_supported(m);
  const bool lusgs = o.precond == FR_PC_LUSGS;
  const bool pmg = o.precond == FR_PC_PMG;
  // small Euler meshes: the JF product of steps with at most kJfDotsMax basis vectors
  // also runs the first DCGS2 pass (one kernel fewer per such step)
  const int jf_dots = dcgs ? residual_dots_blocks(d) : 0;
  volatile GmStatus* hstat = (volatile GmStatus*)d->h_pinned;
  GmStatus* dstat = (GmStatus*)d->d_pinned;
  // The host runs ahead of the GPU and stops enqueueing once the mapped status shows a
  // stop (kernels enqueued after a stop return at once).  An event recorded after every
  // fourth step bounds the lead to about eight steps: an event per step cost about 5 us
  // of GPU idle time each on small meshes.  Restart decisions are taken on the device
  // (k_gm_cycle_end): the next cycle is enqueued behind the current one without a host
  // round trip and does nothing if the solve has ended.  Every cycle but the last runs
  // all m steps (an early stop ends the solve), so cycle c starts after c m iterations.
  hstat->stop = 0;
  hstat->j = 0;
  for (int c = 0; c * m < max_iters; ++c) {
    const int budget = std::min(m, max_iters - c * m);
    FR_HIP(launch_gm_start(W.st, beta2, o.rtol, ref, m, dstat, W.V, c == 0 ? rsrc : W.r, n, c == 0, s));
    for (int j = 0; j < budget; ++j) {
      if (j >= 8 && j % 4 == 0) FR_HIP(hipEventSynchronize(d->ev[(j / 4 - 2) & 3]));  // step j - 5 done
      if (hstat->stop) break;
      double* vj = W.V + (size_t)j * n;
      double* zj = W.Z + (size_t)j * n;
      const int* skip = &W.st->stop;
      // z_j = M^{-1} v_j; for j >= 1 the same kernel first runs the Givens update of step
      // j - 1 and forms v_j = w / h_{j,j-1} on the fly.  The partial sums of ||z_j||^2 go
      // to their own slot, past the rows of both orthogonalisation passes (the JF product
      // that reads them may write the first pass's rows meanwhile).
      double* zpart = W.partials + kPartZ;
      int np = 0;
      if (pmg) {
        const GivensIn gv{W.st, dcgs ? dcgs2_norm_partials(W.partials) : W.partials, cgs_blocks(n), m, dcgs ? 1 : 0};
        fr_status ps = j == 0 ? pmg_apply(d, factors, prec, mg, ra, vj, nullptr, nullptr, zj, W, zpart, &np, skip, s)
                              : pmg_apply(d, factors, prec, mg, ra, W.w, &gv, vj, zj, W, zpart, &np, skip, s);
        if (ps != FR_OK) return ps;
      } else if (lusgs) {
        // LU-SGS: its passes leave their partial sums in the ||z||^2 slot in turn (each
        // read by the next kernel), the last one ||z_j||^2
        const GivensIn gv{W.st, dcgs ? dcgs2_norm_partials(W.partials) : W.partials, cgs_blocks(n), m, dcgs ? 1 : 0};
        fr_status ls = j == 0 ? lusgs_apply(d, factors, prec, ra, vj, nullptr, nullptr, zj, W, zpart, &np, skip,
                                            nullptr, s)
                              : lusgs_apply(d, factors, prec, ra, W.w, &gv, vj, zj, W, zpart, &np, skip, nullptr, s);
        if (ls != FR_OK) return ls;
      } else if (j == 0) {
        FR_HIP(launch_ejacobi_solve(d, factors, prec, vj, nullptr, nullptr, zj, zpart, &np, nullptr, skip, s));
      } else {
        // finish step j - 1, then v_j = w / ||w||
        const GivensIn gv{W.st, dcgs ? dcgs2_norm_partials(W.partials) : W.partials, cgs_blocks(n), m, dcgs ? 1 : 0};
        FR_HIP(launch_ejacobi_solve(d, factors, prec, W.w, &gv, vj, zj, zpart, &np, nullptr, skip, s));
      }
      ResArgs a1 = ra;
      a1.nrm2_part = zpart;  // ||z_j||^2 added by the product itself
      a1.nrm2_nb = np;
      a1.V = zj;
      a1.out = W.w;
      a1.skip = skip;
      const bool fused_dots = jf_dots > 0 && j + 1 <= kJfDotsMax;
      if (fused_dots) {
        a1.dV = W.V;
        a1.dnv = j + 1;
        a1.dpart = W.partials;
      }
      FR_HIP(launch_residual(d, 1, a1, s));
      if (fused_dots)
        FR_HIP(launch_dcgs2_update(W.V, j + 1, W.w, W.partials, jf_dots, W.st, m, n, s));
      else if (dcgs)
        FR_HIP(launch_arnoldi_dcgs2(W.V, j + 1, W.w, W.partials, W.st, m, n, s));
      else
        FR_HIP(launch_arnoldi_cgs2(W.V, j + 1, W.w, W.partials, W.st, m, n, s));
      if (j % 4 == 3) FR_HIP(hipEventRecord(d->ev[(j / 4) & 3], s));
    }
    // the Givens update of the cycle's last column (returns at once after a stop)
    if (dcgs)
      FR_HIP(launch_dcgs2_last(W.st, W.partials, cgs_blocks(n), m, s));
    else
      FR_HIP(launch_givens(W.st, W.partials, cgs_blocks(n), m, s));
    // y and x += Z y (skipped after NaN), then the true residual r = b - A x for a
    // restart (skipped once converged or NaN), then the device's decision
    int nbx = 0;
    FR_HIP(launch_gm_update_x(x, W.Z, m, W.st, n, W.partials, &nbx, s));
    const int* done = &W.st->done;
    ResArgs a2 = ra;
    a2.nrm2_part = W.partials;  // ||x||^2 from the update's partial sums
    a2.nrm2_nb = nbx;
    a2.V = x;
    a2.B = b;
    a2.out = W.r;
    a2.skip = done;
    if (jf_dots > 0) {
      // small Euler meshes: the residual kernel leaves ||r||^2 per tile, the decision adds them
      a2.opart = W.partials + kPartSecond;
      FR_HIP(launch_residual(d, 2, a2, s));
      FR_HIP(launch_gm_cycle_end_parts(W.st, beta2, a2.opart, jf_dots, max_iters, dcgs ? 1 : 0, s));
    } else {
      FR_HIP(launch_residual(d, 2, a2, s));
      FR_HIP(launch_norm2(W.r, n, W.partials, beta2, done, s));
      FR_HIP(launch_gm_cycle_end(W.st, beta2, max_iters, dcgs ? 1 : 0, s));
    }
    if (hstat->stop) break;  // the solve has ended, or its stop is on the way
  }
  GmState::Final fz;
  rs = read_sync(d, &fz, (const char*)W.st + offsetof(GmState, fz), sizeof(fz), s);
  if (rs != FR_OK) return rs;
  S.iters = fz.iters;
  S.residual_evals += fz.evals;
  if (lusgs) S.residual_evals += 2L * fz.steps;  // the two products of every LU-SGS application
  if (pmg) S.residual_evals += (long)pmg_products(mg) * fz.steps;
  S.restarts = fz.restarts;
  S.r_final = fz.r_final;
  S.r_ref = fz.r_ref;
  const fr_status result = fz.fin ? (fr_status)fz.result : FR_NOTCONV;
  S.converged = result == FR_OK ? 1 : 0;
  *stats = S;
  return result;
}

// ---------------------------------------------------------------- time steps
namespace {

struct StepBufs {
  GmWork gw;
  void* pc;
  double* vec[kStepVecs];
};

StepBufs carve_step(const fr_disc* d, void* work, int m, int precision) {
  Carver c(work);
  StepBufs b{};
  b.gw = carve_gmres(c, d, m);
  b.pc = c.take(fr_ejacobi_bytes(d, precision));
  for (int i = 0; i < kStepVecs; ++i) b.vec[i] = (double*)c.take(sizeof(double) * d->ndof);
  return b;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

fr_status residual_into(const fr_disc* d, const double* U, double* R, double* grad, hipStream_t s) {
  ResArgs a{};
  a.U = U;
  a.out = R;
  a.grad = grad;
  FR_HIP(launch_residual(d, 0, a, s));
  return FR_OK;
}

fr_status lincomb(double* y, std::initializer_list<std::pair<const double*, double>> terms, size_t n,
                  hipStream_t s) {
  const double* xs[8];
  double cs[8];
  int k = 0;
  for (auto& t : terms) {
    xs[k] = t.first;
    cs[k] = t.second;
    ++k;
  }
  FR_HIP(launch_lincomb(y, k, xs, cs, n, s));
  return FR_OK;
}

fr_status lincomb_v(double* y, int k, const double* const* xs, const double* cs, size_t n, hipStream_t s) {
  FR_HIP(launch_lincomb(y, k, xs, cs, n, s));
  return FR_OK;
}

#define FR_TRY(expr)                 \
  do {                               \
    fr_status st_ = (expr);          \
    if (st_ < 0) return st_;         \
  } while (0)

// PTC for F(q) = (q - cst)/(omega dt) - R(q) = 0, in place on q; Rq holds R(q) on entry
// (if rq_valid) and on exit.  q_alt (may be null): a second starting point (the learned
// guess); PTC starts from it when its ||F|| is below that of q, and the stopping test
// stays relative to ||F(q)|| either way.  R_alt: scratch for R(q_alt).
fr_status ptc_solve(const fr_disc* d, const double* cst, double omega_dt, double dt, double* q, double* Rq,
                    bool rq_valid, const fr_solver_opts& o, StepBufs& B, fr_step_stats* st, hipStream_t s,
                    const double* q_alt = nullptr, double* R_alt = nullptr) {
  const size_t n = d->ndof;
  double* negF = B.vec[9];
  double* dq = B.vec[10];
  if (!rq_valid) {
    FR_TRY(residual_into(d, q, Rq, B.gw.grad, s));
    st->residual_evals++;
  }
  const double iw = 1.0 / omega_dt;
  FR_TRY(lincomb(negF, {{cst, iw}, {q, -iw}, {Rq, 1.0}}, n, s));
  double nF = 0.0;
  FR_TRY(device_norm(d, negF, B.gw.partials, B.gw.scal + 2, &nF, s));
  const double nF0 = nF;
  if (q_alt != nullptr) {
    FR_TRY(residual_into(d, q_alt, R_alt, B.gw.grad, s));
    st->residual_evals++;
    FR_TRY(lincomb(dq, {{cst, iw}, {q_alt, -iw}, {R_alt, 1.0}}, n, s));
    double nFa = 0.0;
    FR_TRY(device_norm(d, dq, B.gw.partials, B.gw.scal + 2, &nFa, s));
    if (nFa < nF) {
      FR_TRY(lincomb(q, {{q_alt, 1.0}}, n, s));
      FR_TRY(lincomb(Rq, {{R_alt, 1.0}}, n, s));
      FR_TRY(lincomb(negF, {{dq, 1.0}}, n, s));
      nF = nFa;
      st->warm_used++;
    } else {
      st->warm_rejected++;
    }
  }
  double dtau = o.dtau_init > 0 ? o.dtau_init : dt;
  double dtau_max = o.dtau_max > 0 ? o.dtau_max : 1e20;
  const int max_ptc = o.max_ptc > 0 ? o.max_ptc : 200;
  const int max_rej = o.max_reject > 0 ? o.max_reject : 30;
  int k = 0, rejects = 0;
  fr_ejacobi pc{B.pc, o.precond_precision, 0.0, nullptr};
  // written so that a NaN norm enters the loop and ends it as FR_ENAN rather than
  // passing the test as converged
  while (!(nF <= o.tol_nl * nF0)) {
    if (!std::isfinite(nF)) return FR_ENAN;
    if (k >= max_ptc) return FR_NOTCONV;
    if (rejects > max_rej) return FR_REJECTED;
    const double shift = 1.0 / dtau + iw;
    FR_HIP(launch_ejacobi_assemble(d, q, shift, pc.d_factors, pc.precision, 1, B.gw.grad, s));
    FR_TRY(lincomb(dq, {}, n, s));
    fr_gmres_stats gs{};
    fr_status g = gmres_core(d, pc.d_factors, pc.precision, q, Rq, shift, negF, dq, true, o.lin, &gs, B.gw, s, false,
                             nullptr);
    if (g < 0) return g;
    st->gmres_iters += gs.iters;
    st->linear_solves++;
    st->residual_evals += gs.residual_evals;
    if (!gs.converged) st->unconverged++;
    if (g == FR_ENAN) return FR_ENAN;
    if (!(gs.r_final <= 0.1 * gs.r_ref)) {
      // the linear solve did not gain one order of magnitude: reject, halve dtau_max
      st->rejections++;
      rejects++;
      dtau_max *= 0.5;
      dtau = std::min(dtau, dtau_max);
      continue;
    }
    FR_TRY(lincomb(q, {{q, 1.0}, {dq, 1.0}}, n, s));
    FR_TRY(residual_into(d, q, Rq, B.gw.grad, s));
    st->residual_evals++;
    FR_TRY(lincomb(negF, {{cst, iw}, {q, -iw}, {Rq, 1.0}}, n, s));
    double nFn = 0.0;
    FR_TRY(device_norm(d, negF, B.gw.partials, B.gw.scal + 2, &nFn, s));
    dtau = (nFn > 0.0) ? std::min(dtau * nF / nFn, dtau_max) : dtau_max;
    nF = nFn;
    ++k;
    st->ptc_iters++;
  }
  return FR_OK;
}

}  // namespace

fr_status row_step_impl(const fr_disc* d, int scheme, double dt, double* U, const fr_solver_opts& o,
                        fr_step_stats* st, void* work, hipStream_t s) {
  const RowScheme* T = row_scheme(scheme);
  const size_t n = d->ndof;
  const double t0 = now_s();
  StepBufs B = carve_step(d, work, o.lin.m, o.precond_precision);
  double* R0 = B.vec[0];
  double* Ui = B.vec[1];
  double* rhs = B.vec[2];
  double** Y = B.vec + 3;  // up to 6 stage vectors: vec[3..8]
  FR_TRY(residual_into(d, U, R0, B.gw.grad, s));
  st->residual_evals++;
  const double shift = 1.0 / (T->gamma * dt);
  FR_HIP(launch_ejacobi_assemble(d, U, shift, B.pc, o.precond_precision, 1, B.gw.grad, s));
  fr_status worst = FR_OK;
  for (int i = 0; i < T->s; ++i) {
    if (i == 0) {
      FR_TRY(lincomb(rhs, {{R0, 1.0}}, n, s));
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
        FR_TRY(lincomb_v(Ui, k, xs, cs, n, s));
        FR_TRY(residual_into(d, Ui, rhs, B.gw.grad, s));
        st->residual_evals++;
      } else {
        FR_TRY(lincomb(rhs, {{R0, 1.0}}, n, s));
      }
      k = 0;
      xs[k] = rhs;
      cs[k++] = 1.0;
      for (int j = 0; j < i; ++j)
        if (T->c[i][j] != 0.0) {
          xs[k] = Y[j];
          cs[k++] = T->c[i][j] / dt;
        }
      if (k > 1) FR_TRY(lincomb_v(rhs, k, xs, cs, n, s));
    }
    // previous increments seen by stage i: (Y_{i-1}, Y_{i-2}), reaching back into the
    // previous step's last two increments for i < 2
    const double* hist_last = o.d_yhist ? o.d_yhist + n : nullptr;
    const double* hist_prev = o.d_yhist ? o.d_yhist : nullptr;
    const double* Y1 = i >= 1 ? Y[i - 1] : hist_last;
    const double* Y2 = i >= 2 ? Y[i - 2] : (i == 1 ? hist_last : hist_prev);
    bool warm = false;
    if (o.warm != nullptr) {
      FR_HIP(mlp_infer(d, &o.warm[i], U, R0, Y1, Y2, dt, Y[i], o.d_mlp_work, s));
      warm = true;
    } else {
      FR_TRY(lincomb(Y[i], {}, n, s));
    }
    fr_gmres_stats gs{};
    int fell = 0;
    fr_status g = gmres_core(d, B.pc, o.precond_precision, U, R0, shift, rhs, Y[i], !warm, o.lin, &gs, B.gw, s,
                             warm, &fell);
    if (g < 0) return g;
    if (warm) {
      st->warm_used += fell ? 0 : 1;
      st->warm_rejected += fell;
    }
    st->gmres_iters += gs.iters;
    st->linear_solves++;
    st->residual_evals += gs.residual_evals;
    if (g != FR_OK) {
      st->unconverged++;
      if (worst == FR_OK || g == FR_ENAN) worst = g;
    }
    if (o.log != nullptr && g == FR_OK) FR_HIP(mlp_log(d, &o.log[i], U, R0, Y1, Y2, Y[i], dt, s));
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
    FR_TRY(lincomb_v(U, k, xs, cs, n, s));
    if (o.d_yhist != nullptr) {
      FR_TRY(lincomb(o.d_yhist, {{Y[T->s - 2], 1.0}}, n, s));
      FR_TRY(lincomb(o.d_yhist + n, {{Y[T->s - 1], 1.0}}, n, s));
    }
  }
  FR_HIP(hipStreamSynchronize(s));
  st->wall_s = now_s() - t0;
  return worst;
}

fr_status esdirk_step_impl(const fr_disc* d, int scheme, double dt, double* U, const fr_solver_opts& o,
                           fr_step_stats* st, void* work, hipStream_t s) {
  const EsdirkScheme* T = esdirk_scheme(scheme);
  const size_t n = d->ndof;
  const double t0 = now_s();
  StepBufs B = carve_step(d, work, o.lin.m, o.precond_precision);
  double** Rj = B.vec;      // vec[0..5]
  double* q = B.vec[6];
  double* cst = B.vec[7];
  FR_TRY(residual_into(d, U, Rj[0], B.gw.grad, s));
  st->residual_evals++;
  FR_TRY(lincomb(q, {{U, 1.0}}, n, s));
  // learned start (warm: one network per implicit stage) and logging: the stage
  // increments q_i - q^n of the two previous stages, reaching back into the previous
  // step's last two (d_yhist) for the first implicit stages
  const bool incs = o.warm != nullptr || o.log != nullptr || o.d_yhist != nullptr;
  double* inc[2] = {B.vec[12], B.vec[13]};  // increment of stage i at inc[i & 1]
  double* cand = B.vec[14];
  double* R_alt = B.vec[8];
  const double* hist_last = o.d_yhist ? o.d_yhist + n : nullptr;
  const double* hist_prev = o.d_yhist ? o.d_yhist : nullptr;
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
    FR_TRY(lincomb_v(cst, k, xs, cs, n, s));
    FR_TRY(lincomb(Rj[i], {{Rj[i - 1], 1.0}}, n, s));  // R(q) at the stage's starting guess q_{i-1}
    const double* Y1 = i >= 2 ? inc[(i - 1) & 1] : hist_last;
    const double* Y2 = i >= 3 ? inc[(i - 2) & 1] : (i == 2 ? hist_last : hist_prev);
    const double* q_alt = nullptr;
    if (o.warm != nullptr) {
      FR_HIP(mlp_infer(d, &o.warm[i - 1], U, Rj[0], Y1, Y2, dt, cand, o.d_mlp_work, s));
      FR_TRY(lincomb(cand, {{U, 1.0}, {cand, 1.0}}, n, s));
      q_alt = cand;
    }
    fr_status p = ptc_solve(d, cst, T->gamma * dt, dt, q, Rj[i], true, o, B, st, s, q_alt, R_alt);
    if (p < 0) return p;
    if (p != FR_OK && worst == FR_OK) worst = p;
    if (p == FR_ENAN || (p != FR_OK && !o.commit_unconverged)) break;  // the step will not be committed
    if (incs) {
      FR_TRY(lincomb(inc[i & 1], {{q, 1.0}, {U, -1.0}}, n, s));
      if (o.log != nullptr && p == FR_OK) FR_HIP(mlp_log(d, &o.log[i - 1], U, Rj[0], Y1, Y2, inc[i & 1], dt, s));
    }
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
    FR_TRY(lincomb_v(U, k, xs, cs, n, s));
    if (o.d_yhist != nullptr) {
      FR_TRY(lincomb(o.d_yhist, {{inc[(T->s - 2) & 1], 1.0}}, n, s));
      FR_TRY(lincomb(o.d_yhist + n, {{inc[(T->s - 1) & 1], 1.0}}, n, s));
    }
  }
  FR_HIP(hipStreamSynchronize(s));
  st->wall_s = now_s() - t0;
  return worst;
}

fr_status bdf2_step_impl(const fr_disc* d, double dt, const double* Unm1, const double* Un, double* Unp1,
                         const fr_solver_opts& o, fr_step_stats* st, void* work, hipStream_t s) {
  const size_t n = d->ndof;
  const double t0 = now_s();
  StepBufs B = carve_step(d, work, o.lin.m, o.precond_precision);
  double* q = B.vec[0];
  double* Rq = B.vec[1];
  double* cst = B.vec[2];
  double omega;
  if (Unm1 == nullptr) {
    omega = 1.0;
    FR_TRY(lincomb(cst, {{Un, 1.0}}, n, s));
  } else {
    omega = 2.0 / 3.0;
    FR_TRY(lincomb(cst, {{Un, 4.0 / 3.0}, {Unm1, -1.0 / 3.0}}, n, s));
  }
  FR_TRY(lincomb(q, {{Un, 1.0}}, n, s));
  // learned start and logging: the increment q^{n+1} - q^n predicted from q^n, R(q^n)
  // and the previous two step increments (d_yhist)
  const bool incs = o.warm != nullptr || o.log != nullptr || o.d_yhist != nullptr;
  const double* Y1 = o.d_yhist ? o.d_yhist + n : nullptr;
  const double* Y2 = o.d_yhist ? o.d_yhist : nullptr;
  double* inc = B.vec[12];
  double* cand = B.vec[14];
  double* R_alt = B.vec[8];
  const double* q_alt = nullptr;
  bool rq_valid = false;
  if (incs) {
    FR_TRY(residual_into(d, q, Rq, B.gw.grad, s));  // R(q^n): features, and PTC's start
    st->residual_evals++;
    rq_valid = true;
  }
  if (o.warm != nullptr) {
    FR_HIP(mlp_infer(d, &o.warm[0], Un, Rq, Y1, Y2, dt, cand, o.d_mlp_work, s));
    FR_TRY(lincomb(cand, {{Un, 1.0}, {cand, 1.0}}, n, s));
    q_alt = cand;
  }
  if (o.log != nullptr) FR_TRY(lincomb(B.vec[13], {{Rq, 1.0}}, n, s));  // R(q^n) kept for the log
  fr_status p = ptc_solve(d, cst, omega * dt, dt, q, Rq, rq_valid, o, B, st, s, q_alt, R_alt);
  if (p < 0) return p;
  if (incs && (p == FR_OK || (o.commit_unconverged && p != FR_ENAN))) {
    FR_TRY(lincomb(inc, {{q, 1.0}, {Un, -1.0}}, n, s));
    if (o.log != nullptr && p == FR_OK) FR_HIP(mlp_log(d, &o.log[0], Un, B.vec[13], Y1, Y2, inc, dt, s));
    if (o.d_yhist != nullptr) {
      FR_TRY(lincomb(o.d_yhist, {{o.d_yhist + n, 1.0}}, n, s));
      FR_TRY(lincomb(o.d_yhist + n, {{inc, 1.0}}, n, s));
    }
  }
  if (p == FR_OK || (o.commit_unconverged && p != FR_ENAN)) FR_TRY(lincomb(Unp1, {{q, 1.0}}, n, s));
  FR_HIP(hipStreamSynchronize(s));
  st->wall_s = now_s() - t0;
  return p;
}

}  // namespace frjf
