// p-multigrid preconditioner (Section 4.5 names it beside element-Jacobi): two FR
// discretisations of one mesh, degree P (fine) and Pc < P (coarse, its own residual and
// element blocks), and a V-cycle with element-Jacobi smoothing on both levels:
//   z  = D^{-1} r,                      then nu1 - 1 sweeps z += D^{-1}(r - A z);
//   rc = Pi (r - A z);   zc = Dc^{-1} rc, then nc - 1 sweeps zc += Dc^{-1}(rc - Ac zc);
//   z += I zc,                          then nu2 sweeps z += D^{-1}(r - A z).
// A, Ac: the Jacobian-free products of the two levels (the coarse one at Uc = Pi U).
// Pi: L2 projection onto degree Pc, (Pi f)_a = (1/w^c_a) sum_b w_b l^c_a(x_b) (exact with
// the fine Gauss rule); I: interpolation of the coarse polynomial, I_ba = l^c_a(x_b);
// both applied per element and variable as tensor products (k_ptransfer).
#include <cmath>

#include "internal.h"
#include "solvers.h"
#include "wavesum.h"

namespace frjf {

struct Transfer1D {
  double T[kMaxN][kMaxN];  // [out][in]
  int nin, nout;
};

// out[v][e][ko] = (add ? base[v][e][ko] : 0) + sum_{bi, ai} T[bo][bi] T[ao][ai] (x1 - x2)[v][e][bi nin + ai]
__global__ void __launch_bounds__(256) k_ptransfer(const Transfer1D t, const double* __restrict__ x1,
                                                   const double* __restrict__ x2, const double* base,
                                                   double* out, int nel, const int* skip) {
  if (skip != nullptr && *skip) return;
  const int nin = t.nin, nout = t.nout, npi = nin * nin, npo = nout * nout;
  const size_t total = (size_t)4 * nel * npo;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const size_t ve = i / npo;  // v nel + e
    const int ko = (int)(i - ve * npo), bo = ko / nout, ao = ko - bo * nout;
    const double* p1 = x1 + ve * npi;
    const double* p2 = x2 != nullptr ? x2 + ve * npi : nullptr;
    double s = 0.0;
    for (int bi = 0; bi < nin; ++bi) {
      double r = 0.0;
      for (int ai = 0; ai < nin; ++ai) {
        const double x = p2 != nullptr ? p1[bi * nin + ai] - p2[bi * nin + ai] : p1[bi * nin + ai];
        r = fma(t.T[ao][ai], x, r);
      }
      s = fma(t.T[bo][bi], r, s);
    }
    out[i] = base != nullptr ? base[i] + s : s;
  }
}

// z = z + t and per-workgroup partial sums of ||z||^2
__global__ void __launch_bounds__(256) k_add_norm(double* __restrict__ z, const double* __restrict__ t, size_t n,
                                                  double* partials, const int* skip) {
  if (skip != nullptr && *skip) return;
  double acc = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double v = z[i] + t[i];
    z[i] = v;
    acc = fma(v, v, acc);
  }
  __shared__ double red[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

static double lagrange_at(const Basis& b, int a, double x) {
  double p = 1.0;
  for (int c = 0; c < b.n; ++c)
    if (c != a) p *= (x - b.x[c]) / (b.x[a] - b.x[c]);
  return p;
}

static Transfer1D restriction_1d(const Basis& f, const Basis& c) {
  Transfer1D t{};
  t.nin = f.n;
  t.nout = c.n;
  for (int a = 0; a < c.n; ++a)
    for (int b = 0; b < f.n; ++b) t.T[a][b] = f.w[b] * lagrange_at(c, a, f.x[b]) / c.w[a];
  return t;
}

static Transfer1D prolongation_1d(const Basis& f, const Basis& c) {
  Transfer1D t{};
  t.nin = c.n;
  t.nout = f.n;
  for (int b = 0; b < f.n; ++b)
    for (int a = 0; a < c.n; ++a) t.T[b][a] = lagrange_at(c, a, f.x[b]);
  return t;
}

static hipError_t transfer(const Transfer1D& t, const double* x1, const double* x2, const double* base, double* out,
                           int nel, const int* skip, hipStream_t s) {
  const size_t total = (size_t)4 * nel * t.nout * t.nout;
  const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_ptransfer, dim3(blocks ? blocks : 1), dim3(256), 0, s, t, x1, x2, base, out, nel, skip);
  return hipGetLastError();
}

static int add_norm_blocks(size_t n) { return (int)std::max<size_t>(1, std::min<size_t>((n + 1023) / 1024, 1024)); }

static hipError_t add_norm(double* z, const double* t, size_t n, double* partials, int* nb, const int* skip,
                           hipStream_t s) {
  *nb = add_norm_blocks(n);
  hipLaunchKernelGGL(k_add_norm, dim3(*nb), dim3(256), 0, s, z, t, n, partials, skip);
  return hipGetLastError();
}

bool pmg_compatible(const fr_disc* f, const fr_pmg* mg) {
  const fr_disc* c = mg != nullptr ? mg->coarse : nullptr;
  return c != nullptr && f->physics == FR_EULER && c->physics == FR_EULER && c->nx == f->nx && c->ny == f->ny &&
         c->p < f->p && c->flux == f->flux && c->phys.gamma == f->phys.gamma && mg->coarse_pc.d_factors != nullptr &&
         mg->d_Uc != nullptr && mg->d_R0c != nullptr && mg->d_work_c != nullptr && mg->nu1 >= 1 && mg->nu2 >= 0 &&
         mg->nc >= 1;
}

fr_status pmg_factor(const fr_disc* f, const double* U, double shift, fr_ejacobi* pc, fr_pmg* mg, double* grad,
                     hipStream_t s) {
  const fr_disc* c = mg->coarse;
  FR_HIP(launch_ejacobi_assemble(f, U, shift, pc->d_factors, pc->precision, 1, grad, s));
  pc->shift = shift;
  const Transfer1D Pi = restriction_1d(f->basis, c->basis);
  FR_HIP(transfer(Pi, U, nullptr, nullptr, mg->d_Uc, f->nel, nullptr, s));
  ResArgs a{};
  a.U = mg->d_Uc;
  a.out = mg->d_R0c;
  FR_HIP(launch_residual(c, 0, a, s));
  FR_HIP(launch_ejacobi_assemble(c, mg->d_Uc, shift, mg->coarse_pc.d_factors, mg->coarse_pc.precision, 1, nullptr,
                                 s));
  mg->coarse_pc.shift = shift;
  return FR_OK;
}

fr_status pmg_apply(const fr_disc* f, const void* factors, int prec, const fr_pmg* mg, const ResArgs& ra,
                    const double* r, const GivensIn* gv, double* r_store, double* z, GmWork& W, double* zpart,
                    int* np, const int* skip, hipStream_t s) {
  const fr_disc* c = mg->coarse;
  const size_t n = f->ndof, nc = c->ndof;
  double* w = W.t[0];   // fine products
  double* t = W.t[1];   // fine smoother corrections
  double* rc = mg->d_work_c;
  double* zc = rc + nc;
  double* wc = zc + nc;
  double* tc = wc + nc;
  double* scal_c = tc + nc;  // coarse ||zc||^2 (large meshes)
  double* part = W.partials + kPartZ;
  const double* rr = (gv != nullptr && r_store != nullptr) ? r_store : r;  // r / ||r|| once stored
  int nb = 0;
  ResArgs a = ra;
  a.out = w;
  a.skip = skip;
  a.dV = nullptr;
  a.opart = nullptr;
  a.B = nullptr;
  // pre-smoothing: z = D^{-1} r (with gv: the Givens update and r / ||r|| first)
  FR_HIP(launch_ejacobi_solve(f, factors, prec, r, gv, r_store, z, part, &nb, nullptr, skip, s));
  for (int k = 1; k < mg->nu1; ++k) {
    a.V = z;
    a.nrm2_part = part;
    a.nrm2_nb = nb;
    FR_HIP(launch_residual(f, 1, a, s));
    const double* xs[2] = {rr, w};
    const double cs[2] = {1.0, -1.0};
    FR_HIP(launch_lincomb(t, 2, xs, cs, n, s));
    FR_HIP(launch_ejacobi_solve(f, factors, prec, t, nullptr, nullptr, w, nullptr, nullptr, nullptr, skip, s));
    FR_HIP(add_norm(z, w, n, part, &nb, skip, s));
  }
  // coarse correction: rc = Pi (r - A z), zc = Dc^{-1} rc (+ sweeps), z += I zc
  a.V = z;
  a.nrm2_part = part;
  a.nrm2_nb = nb;
  FR_HIP(launch_residual(f, 1, a, s));
  const Transfer1D Pi = restriction_1d(f->basis, c->basis), I = prolongation_1d(f->basis, c->basis);
  FR_HIP(transfer(Pi, rr, w, nullptr, rc, f->nel, skip, s));
  int nbc = 0;
  FR_HIP(launch_ejacobi_solve(c, mg->coarse_pc.d_factors, mg->coarse_pc.precision, rc, nullptr, nullptr, zc, part,
                              &nbc, nullptr, skip, s));
  for (int k = 1; k < mg->nc; ++k) {
    ResArgs ac{};
    ac.U = mg->d_Uc;
    ac.R0 = mg->d_R0c;
    ac.V = zc;
    ac.out = wc;
    ac.nrm2 = scal_c;
    ac.nrm2_part = part;
    ac.nrm2_nb = nbc;
    ac.eps = ra.eps;
    ac.eps_mode = ra.eps_mode;
    ac.shift = ra.shift;
    ac.skip = skip;
    FR_HIP(launch_residual(c, 1, ac, s));  // wc = Ac zc
    const double* xs[2] = {rc, wc};
    const double cs[2] = {1.0, -1.0};
    FR_HIP(launch_lincomb(tc, 2, xs, cs, nc, s));
    FR_HIP(launch_ejacobi_solve(c, mg->coarse_pc.d_factors, mg->coarse_pc.precision, tc, nullptr, nullptr, wc,
                                nullptr, nullptr, nullptr, skip, s));
    FR_HIP(add_norm(zc, wc, nc, part, &nbc, skip, s));
  }
  FR_HIP(transfer(I, zc, nullptr, z, z, f->nel, skip, s));  // z += I zc
  // post-smoothing; the last kernel leaves the partial sums of ||z||^2 for the caller
  if (mg->nu2 == 0) {
    FR_HIP(launch_norm2_parts(z, n, zpart, np, skip, s));
    return FR_OK;
  }
  FR_HIP(launch_norm2_parts(z, n, part, &nb, skip, s));
  for (int k = 0; k < mg->nu2; ++k) {
    a.V = z;
    a.nrm2_part = part;
    a.nrm2_nb = nb;
    FR_HIP(launch_residual(f, 1, a, s));
    const double* xs[2] = {rr, w};
    const double cs[2] = {1.0, -1.0};
    FR_HIP(launch_lincomb(t, 2, xs, cs, n, s));
    FR_HIP(launch_ejacobi_solve(f, factors, prec, t, nullptr, nullptr, w, nullptr, nullptr, nullptr, skip, s));
    FR_HIP(add_norm(z, w, n, k + 1 == mg->nu2 ? zpart : part, k + 1 == mg->nu2 ? np : &nb, skip, s));
  }
  return FR_OK;
}

// Jacobian-free products of one application: (nu1 - 1) + 1 + nu2 fine, nc - 1 coarse
// (coarse products cost (Pc+1)^2 / (P+1)^2 of a fine one; counted as whole ones)
int pmg_products(const fr_pmg* mg) { return mg->nu1 + mg->nu2 + (mg->nc - 1); }

}  // namespace frjf
