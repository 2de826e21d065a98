// Internal interfaces of the host drivers.
#pragma once
#include "internal.h"

namespace frjf {

struct RowScheme {
  int s;
  double gamma;
  double a[6][6], c[6][6], m[6];
};
struct EsdirkScheme {
  int s;
  double gamma;
  double a[6][6], b[6];
};
const RowScheme* row_scheme(int id);
const EsdirkScheme* esdirk_scheme(int id);

struct GmWork {
  double* grad;  // BR1 gradient traces (Navier-Stokes only)
  GmState* st;
  double* scal;
  double* partials;
  double* V;
  double* Z;
  double* w;
  double* r;
  double* t[3];  // LU-SGS: the forward sweep's y, the black part of y, a product
};

struct Carver {
  char* p;
  explicit Carver(void* base);
  void* take(size_t bytes);
};

size_t gmres_bytes(const fr_disc* d, int m);
size_t ns_trace_bytes(const fr_disc* d);
size_t small_bytes(const fr_disc* d);
size_t partials_count(const fr_disc* d);
GmWork carve_gmres(Carver& c, const fr_disc* d, int m);
fr_status device_norm(const fr_disc* d, const double* x, double* partials, double* dev_out,
                      double* host_out, hipStream_t s);

// z = M^{-1} r by LU-SGS (see ejacobi.hip): three passes over the element blocks and two
// Jacobian-free products; with gv, r is first scaled by 1/||r|| (from gv's partials) and
// stored to r_store.  ra: the JF product's arguments (U, R0, shift, eps).  Leaves the
// partial sums of ||z||^2 in zpart (*np of them); counts its products in *evals.
fr_status lusgs_apply(const fr_disc* d, const void* factors, int prec, const ResArgs& ra, const double* r,
                      const GivensIn* gv, double* r_store, double* z, GmWork& W, double* zpart, int* np,
                      const int* skip, long* evals, hipStream_t s);
// p-multigrid (pmg.hip): compatibility of the two levels, their factorisation, and one
// V-cycle z = M^{-1} r with the same conventions as lusgs_apply; pmg_products: the
// Jacobian-free products of one application.
bool pmg_compatible(const fr_disc* fine, const fr_pmg* mg);
fr_status pmg_factor(const fr_disc* fine, const double* U, double shift, fr_ejacobi* pc, fr_pmg* mg, double* grad,
                     hipStream_t s);
fr_status pmg_apply(const fr_disc* fine, const void* factors, int prec, const fr_pmg* mg, const ResArgs& ra,
                    const double* r, const GivensIn* gv, double* r_store, double* z, GmWork& W, double* zpart,
                    int* np, const int* skip, hipStream_t s);
int pmg_products(const fr_pmg* mg);
fr_status gmres_core(const fr_disc* d, const void* factors, int prec, const double* U, const double* R0,
                     double shift, const double* b, double* x, bool x_is_zero, const fr_gmres_opts& o,
                     fr_gmres_stats* stats, GmWork& W, hipStream_t s, bool plain_fallback = false,
                     int* fell_back = nullptr, const fr_pmg* mg = nullptr);
fr_status row_step_impl(const fr_disc* d, int scheme, double dt, double* U, const fr_solver_opts& o,
                        fr_step_stats* st, void* work, hipStream_t s);
fr_status esdirk_step_impl(const fr_disc* d, int scheme, double dt, double* U, const fr_solver_opts& o,
                           fr_step_stats* st, void* work, hipStream_t s);
fr_status bdf2_step_impl(const fr_disc* d, double dt, const double* Unm1, const double* Un, double* Unp1,
                         const fr_solver_opts& o, fr_step_stats* st, void* work, hipStream_t s);

// Implicit steps on the 3D path (implicit3d.hip).
size_t fr3d_step_bytes(const fr3d_disc* d, int m);
size_t fr3d_block_bytes(const fr3d_disc* d);
fr_status fr3d_assemble_impl(const fr3d_disc* d, const double* U, double shift, double* blocks, void* work,
                             hipStream_t s);
fr_status fr3d_factor_impl(const fr3d_disc* d, const double* U, double shift, double* inv, void* work,
                           hipStream_t s);
fr_status fr3d_apply_impl(const fr3d_disc* d, const double* inv, const double* r, double* z, hipStream_t s);
fr_status fr3d_gmres_impl(const fr3d_disc* d, const double* inv, const double* U, const double* R0, double shift,
                          const double* b, double* x, const fr_gmres_opts& o, fr_gmres_stats* st, void* work,
                          hipStream_t s);
fr_status fr3d_row_impl(const fr3d_disc* d, int scheme, double dt, double* U, const fr_solver_opts& o,
                        fr_step_stats* st, void* work, hipStream_t s);
fr_status fr3d_esdirk_impl(const fr3d_disc* d, int scheme, double dt, double* U, const fr_solver_opts& o,
                           fr_step_stats* st, void* work, hipStream_t s);
fr_status fr3d_bdf2_impl(const fr3d_disc* d, double dt, const double* Unm1, const double* Un, double* Unp1,
                         const fr_solver_opts& o, fr_step_stats* st, void* work, hipStream_t s);

}  // namespace frjf
