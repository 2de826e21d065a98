// C ABI entry points (include/frjf.h): argument checks, workspace carving and
// dispatch to the kernels and host drivers.
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>
#include <algorithm>
#include <mutex>

#include "internal.h"
#include "solvers.h"

namespace frjf {

static thread_local std::string g_err;

fr_status set_error(fr_status st, const std::string& msg) {
  g_err = msg;
  return st;
}
void clear_error() { g_err.clear(); }

}  // namespace frjf

using namespace frjf;

// ---------------------------------------------------------------- static scratch
// Device memory of fr_jf_matvec_noalloc: the RMS norm's partial sums and its finished
// value, then (Navier-Stokes) the BR1 gradient traces.  Every GPU the library runs on
// holds its own copy until the process ends; calls on one GPU share it.  In host code
// the array's name is only a stand-in: its device address comes from
// hipGetSymbolAddress, once per device (scratch_address).
constexpr size_t kScratchBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr size_t kScratchScalBytes = 256;                              // ||v||^2
constexpr size_t kScratchPartBytes = sizeof(double) * kRedBlocks;     // its partial sums
constexpr size_t kScratchTraceOff = kScratchScalBytes + kScratchPartBytes;

static std::mutex g_scratch_mu;
static void* g_scratch_addr[256];

// Device address of `scratch` on `device` (current when called), looked up on first use.
static hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= 256) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_addr[device] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

#define CHECK(cond, msg)                                   \
  do {                                                     \
    if (!(cond)) return set_error(FR_EINVAL, msg);         \
  } while (0)

static inline hipStream_t S(fr_stream s) { return (hipStream_t)s; }

extern "C" {

const char* fr_last_error(void) { return g_err.c_str(); }

fr_status fr_disc_create(const fr_disc_desc* desc, fr_disc** out) {
  clear_error();
  CHECK(desc != nullptr && out != nullptr, "fr_disc_create: null argument");
  CHECK(desc->p >= 2 && desc->p <= 6, "fr_disc_create: p must be 2 .. 6");
  CHECK(desc->nx >= 2 && desc->ny >= 2, "fr_disc_create: nx and ny must be >= 2");
  CHECK(desc->physics == FR_EULER || desc->physics == FR_NS_BR1, "fr_disc_create: bad physics");
  CHECK(desc->flux == FR_RUSANOV || desc->flux == FR_ROE, "fr_disc_create: bad flux");
  CHECK(desc->d_nodes != nullptr, "fr_disc_create: d_nodes is null");
  CHECK(desc->gamma > 1.0 && desc->rgas > 0.0, "fr_disc_create: gamma must exceed 1 and R be positive");
  CHECK((size_t)desc->nx * desc->ny < (1u << 30), "fr_disc_create: mesh too large");
  if (desc->physics == FR_NS_BR1) {
    CHECK(desc->p <= 4, "fr_disc_create: Navier-Stokes supports p = 2, 3, 4");
    CHECK(desc->mu >= 0.0 && desc->prandtl > 0.0, "fr_disc_create: mu >= 0 and Pr > 0 required");
  }
  CHECK(desc->viscous == FR_BR1 || desc->viscous == FR_BR2, "fr_disc_create: bad viscous scheme");
  for (int b : {desc->bc_south, desc->bc_north}) {
    CHECK(b == FR_BC_PERIODIC || b == FR_BC_WALL || b == FR_BC_FARFIELD, "fr_disc_create: bad boundary");
    CHECK(b == FR_BC_PERIODIC || desc->physics == FR_NS_BR1,
          "fr_disc_create: wall and far-field boundaries need the Navier-Stokes physics");
  }
  if (desc->bc_south == FR_BC_FARFIELD || desc->bc_north == FR_BC_FARFIELD) {
    const double* q = desc->q_far;
    const double pf = (desc->gamma - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0]);
    CHECK(q[0] > 0.0 && pf > 0.0, "fr_disc_create: far-field state needs rho > 0 and p > 0");
  }
  fr_disc* d = new fr_disc{};
  d->nx = desc->nx;
  d->ny = desc->ny;
  d->p = desc->p;
  d->n = desc->p + 1;
  d->np = d->n * d->n;
  d->nb = 4 * d->np;
  d->nel = desc->nx * desc->ny;
  d->physics = desc->physics;
  d->flux = desc->flux;
  d->visc = desc->viscous;
  d->bc_south = desc->bc_south;
  d->bc_north = desc->bc_north;
  for (int v = 0; v < 4; ++v) d->qfar[v] = desc->q_far[v];
  d->ndof = (size_t)4 * d->nel * d->np;
  d->phys.gamma = desc->gamma;
  d->phys.rgas = desc->rgas;
  d->phys.mu = desc->mu;
  d->phys.prandtl = desc->prandtl;
  d->phys.cp_over_pr = desc->physics == FR_NS_BR1 ? desc->gamma * desc->rgas / (desc->gamma - 1.0) / desc->prandtl : 0.0;
  d->basis = make_basis(desc->p);
  d->nodes = desc->d_nodes;
  hipError_t e = hipGetDevice(&d->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&d->ncu, hipDeviceAttributeMultiprocessorCount, d->device);
  if (e == hipSuccess) e = hipHostMalloc(&d->h_pinned, 4096, hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess) e = hipHostGetDevicePointer(&d->d_pinned, d->h_pinned, 0);
  for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&d->ev[i], hipEventDisableTiming);
  if (e == hipSuccess) e = scratch_address(d->device, &d->d_scratch);
  if (e != hipSuccess) {
    delete d;
    return set_error(FR_EHIP, std::string("fr_disc_create: ") + hipGetErrorString(e));
  }
  *out = d;
  return FR_OK;
}

void fr_disc_destroy(fr_disc* d) {
  if (d == nullptr) return;
  for (int i = 0; i < 4; ++i)
    if (d->ev[i]) (void)hipEventDestroy(d->ev[i]);
  if (d->h_pinned) (void)hipHostFree(d->h_pinned);
  delete d;
}

size_t fr_ndof(const fr_disc* d) { return d ? d->ndof : 0; }

size_t fr_ejacobi_bytes(const fr_disc* d, int precision) {
  if (d == nullptr) return 0;
  const size_t es = precision == FR_F32 ? sizeof(float) : sizeof(double);
  return (size_t)d->nel * d->nb * d->nb * es;
}

size_t fr_workspace_bytes(const fr_disc* d, int what, int m, int precision) {
  if (d == nullptr) return 0;
  const size_t vec = ((sizeof(double) * d->ndof) + 255) & ~(size_t)255;
  const size_t tr = (ns_trace_bytes(d) + 255) & ~(size_t)255;
  switch (what) {
    case FR_WS_RESIDUAL: return tr;
    case FR_WS_MATVEC: return tr + small_bytes(d);
    case FR_WS_GMRES: return gmres_bytes(d, m < 1 ? 1 : m);
    case FR_WS_STEP:
      return gmres_bytes(d, m < 1 ? 1 : m) + ((fr_ejacobi_bytes(d, precision) + 255) & ~(size_t)255) +
             kStepVecs * vec;
  }
  return 0;
}

static double* ns_traces(const fr_disc* d, void* work) { return d->physics == FR_NS_BR1 ? (double*)work : nullptr; }

fr_status fr_solution_points(const fr_disc* d, double* xy, fr_stream s) {
  clear_error();
  CHECK(d && xy, "fr_solution_points: null argument");
  FR_HIP(launch_solution_points(d, xy, S(s)));
  return FR_OK;
}

fr_status fr_residual(const fr_disc* d, const double* U, double* R, void* work, fr_stream s) {
  clear_error();
  CHECK(d && U && R, "fr_residual: null argument");
  CHECK(U != R, "fr_residual: U and R alias");
  CHECK(d->physics == FR_EULER || work != nullptr, "fr_residual: Navier-Stokes needs a workspace");
  ResArgs a{};
  a.U = U;
  a.out = R;
  a.grad = ns_traces(d, work);
  FR_HIP(launch_residual(d, 0, a, S(s)));
  return FR_OK;
}

fr_status fr_jf_matvec(const fr_disc* d, const double* U, const double* R0, const double* v, double shift, double eps,
                       int eps_mode, double* Av, void* work, fr_stream s) {
  clear_error();
  CHECK(d && U && R0 && v && Av && work, "fr_jf_matvec: null argument");
  CHECK(Av != U && Av != R0 && Av != v, "fr_jf_matvec: output aliases an input");
  CHECK(eps_mode == FR_EPS_ABS || eps_mode == FR_EPS_RMS, "fr_jf_matvec: bad eps_mode");
  CHECK(eps > 0.0, "fr_jf_matvec: eps must be positive");
  Carver c(work);
  double* tr = (double*)c.take(ns_trace_bytes(d));
  double* scal = (double*)c.take(256);
  double* partials = (double*)c.take(sizeof(double) * partials_count(d));
  if (eps_mode == FR_EPS_RMS) FR_HIP(launch_norm2(v, d->ndof, partials, scal, nullptr, S(s)));
  ResArgs a{};
  a.U = U;
  a.V = v;
  a.R0 = R0;
  a.out = Av;
  a.nrm2 = scal;
  a.eps = eps;
  a.eps_mode = eps_mode;
  a.shift = shift;
  a.grad = d->physics == FR_NS_BR1 ? tr : nullptr;
  FR_HIP(launch_residual(d, 1, a, S(s)));
  return FR_OK;
}

fr_status fr_jf_matvec_noalloc(const fr_disc* d, const double* U, const double* R0, const double* v, double shift,
                               double eps, int eps_mode, double* Av, fr_stream s) {
  clear_error();
  CHECK(d && U && R0 && v && Av, "fr_jf_matvec_noalloc: null argument");
  CHECK(Av != U && Av != R0 && Av != v, "fr_jf_matvec_noalloc: output aliases an input");
  CHECK(eps_mode == FR_EPS_ABS || eps_mode == FR_EPS_RMS, "fr_jf_matvec_noalloc: bad eps_mode");
  CHECK(eps > 0.0, "fr_jf_matvec_noalloc: eps must be positive");
  if (d->d_scratch == nullptr) return set_error(FR_EHIP, "fr_jf_matvec_noalloc: no scratch address for the device");
  const size_t tr = ns_trace_bytes(d);
  if (kScratchTraceOff + tr > kScratchBytes)
    return set_error(FR_ESIZE, "fr_jf_matvec_noalloc: the mesh's BR1 gradient traces (" + std::to_string(tr) +
                                   " bytes) exceed the static scratch (" +
                                   std::to_string(kScratchBytes - kScratchTraceOff) + " bytes)");
  char* base = (char*)d->d_scratch;
  double* scal = (double*)base;
  double* partials = (double*)(base + kScratchScalBytes);
  if (eps_mode == FR_EPS_RMS) FR_HIP(launch_norm2(v, d->ndof, partials, scal, nullptr, S(s)));
  ResArgs a{};
  a.U = U;
  a.V = v;
  a.R0 = R0;
  a.out = Av;
  a.nrm2 = scal;
  a.eps = eps;
  a.eps_mode = eps_mode;
  a.shift = shift;
  a.grad = d->physics == FR_NS_BR1 ? (double*)(base + kScratchTraceOff) : nullptr;
  FR_HIP(launch_residual(d, 1, a, S(s)));
  return FR_OK;
}

fr_status fr_ejacobi_assemble(const fr_disc* d, const double* U, double shift, double* blocks, void* work,
                              fr_stream s) {
  clear_error();
  CHECK(d && U && blocks, "fr_ejacobi_assemble: null argument");
  CHECK(d->physics == FR_EULER || work != nullptr, "fr_ejacobi_assemble: Navier-Stokes needs a workspace");
  FR_HIP(launch_ejacobi_assemble(d, U, shift, blocks, FR_F64, 0, ns_traces(d, work), S(s)));
  return FR_OK;
}

fr_status fr_ejacobi_factor(const fr_disc* d, const double* U, double shift, fr_ejacobi* pc, void* work,
                            fr_stream s) {
  clear_error();
  CHECK(d && U && pc && pc->d_factors, "fr_ejacobi_factor: null argument");
  CHECK(pc->precision == FR_F64 || pc->precision == FR_F32, "fr_ejacobi_factor: bad precision");
  CHECK(d->physics == FR_EULER || work != nullptr, "fr_ejacobi_factor: Navier-Stokes needs a workspace");
  FR_HIP(launch_ejacobi_assemble(d, U, shift, pc->d_factors, pc->precision, 1, ns_traces(d, work), S(s)));
  pc->shift = shift;
  return FR_OK;
}

fr_status fr_ejacobi_factor_blocks(const fr_disc* d, const double* blocks, fr_ejacobi* pc, fr_stream s) {
  clear_error();
  CHECK(d && blocks && pc && pc->d_factors, "fr_ejacobi_factor_blocks: null argument");
  CHECK(pc->precision == FR_F64 || pc->precision == FR_F32, "fr_ejacobi_factor_blocks: bad precision");
  CHECK((const void*)blocks != pc->d_factors || pc->precision == FR_F64,
        "fr_ejacobi_factor_blocks: in-place inversion needs FR_F64");
  FR_HIP(launch_ejacobi_invert_blocks(d, blocks, pc->d_factors, pc->precision, S(s)));
  return FR_OK;
}

fr_status fr_ejacobi_solve(const fr_disc* d, const fr_ejacobi* pc, const double* r, double* z, fr_stream s) {
  clear_error();
  CHECK(d && pc && pc->d_factors && r && z, "fr_ejacobi_solve: null argument");
  CHECK(r != z, "fr_ejacobi_solve: r and z alias");
  CHECK(pc->precision == FR_F64 || pc->precision == FR_F32, "fr_ejacobi_solve: bad precision");
  FR_HIP(launch_ejacobi_solve(d, pc->d_factors, pc->precision, r, nullptr, nullptr, z, nullptr, nullptr, nullptr,
                              nullptr, S(s)));
  return FR_OK;
}

static fr_status check_gmres_opts(const fr_gmres_opts* o) {
  CHECK(o != nullptr, "null GMRES options");
  CHECK(o->m >= 1 && o->m <= kMaxM, "GMRES restart m must be in 1..64");
  CHECK(o->rtol >= 0.0, "GMRES rtol must be >= 0");
  CHECK(o->eps_mode == FR_EPS_ABS || o->eps_mode == FR_EPS_RMS, "bad eps_mode");
  CHECK(o->precond == FR_PC_EJACOBI || o->precond == FR_PC_LUSGS || o->precond == FR_PC_PMG, "bad precond");
  return FR_OK;
}

fr_status fr_lusgs_apply(const fr_disc* d, const fr_ejacobi* pc, const double* U, const double* R0, double shift,
                         double eps, int eps_mode, const double* r, double* z, void* work, fr_stream s) {
  clear_error();
  CHECK(d && pc && pc->d_factors && U && R0 && r && z && work, "fr_lusgs_apply: null argument");
  CHECK(z != r && z != U && z != R0, "fr_lusgs_apply: z aliases an input");
  CHECK(pc->precision == FR_F64 || pc->precision == FR_F32, "fr_lusgs_apply: bad precision");
  CHECK(eps_mode == FR_EPS_ABS || eps_mode == FR_EPS_RMS, "fr_lusgs_apply: bad eps_mode");
  CHECK(eps > 0.0, "fr_lusgs_apply: eps must be positive");
  CHECK(d->physics == FR_EULER && !(d->nx & 1) && !(d->ny & 1),
        "fr_lusgs_apply: Euler meshes with even nx and ny only");
  Carver cv(work);
  GmWork W = carve_gmres(cv, d, 1);
  ResArgs ra{};
  ra.U = U;
  ra.R0 = R0;
  ra.eps = eps;
  ra.eps_mode = eps_mode;
  ra.shift = shift;
  ra.nrm2 = W.scal;
  int np = 0;
  return lusgs_apply(d, pc->d_factors, pc->precision, ra, r, nullptr, nullptr, z, W, W.partials + kPartZ, &np,
                     nullptr, nullptr, S(s));
}

fr_status fr_gmres_solve(const fr_disc* d, const fr_ejacobi* pc, const double* U, const double* R0, double shift,
                         const double* b, double* x, const fr_gmres_opts* opts, fr_gmres_stats* stats, void* work,
                         fr_stream s) {
  clear_error();
  CHECK(d && pc && pc->d_factors && U && R0 && b && x && stats && work, "fr_gmres_solve: null argument");
  fr_status c = check_gmres_opts(opts);
  if (c != FR_OK) return c;
  CHECK(x != b && x != U && x != R0, "fr_gmres_solve: x aliases an input");
  Carver cv(work);
  GmWork W = carve_gmres(cv, d, opts->m);
  return gmres_core(d, pc->d_factors, pc->precision, U, R0, shift, b, x, false, *opts, stats, W, S(s), false,
                    nullptr, pc->mg);
}

fr_status fr_pmg_factor(const fr_disc* d, const double* U, double shift, fr_ejacobi* pc, fr_pmg* mg, void* work,
                        fr_stream s) {
  clear_error();
  CHECK(d && U && pc && pc->d_factors && mg, "fr_pmg_factor: null argument");
  CHECK(pc->precision == FR_F64 || pc->precision == FR_F32, "fr_pmg_factor: bad precision");
  CHECK(mg->coarse_pc.precision == FR_F64 || mg->coarse_pc.precision == FR_F32, "fr_pmg_factor: bad coarse precision");
  CHECK(pmg_compatible(d, mg), "fr_pmg_factor: levels do not match (same mesh and flux, Euler, coarse p < fine p, "
                               "buffers set, nu1 >= 1, nu2 >= 0, nc >= 1)");
  (void)work;
  fr_status st = pmg_factor(d, U, shift, pc, mg, nullptr, S(s));
  if (st == FR_OK) pc->mg = mg;
  return st;
}

fr_status fr_pmg_apply(const fr_disc* d, const fr_ejacobi* pc, const double* U, const double* R0, double shift,
                       double eps, int eps_mode, const double* r, double* z, void* work, fr_stream s) {
  clear_error();
  CHECK(d && pc && pc->d_factors && U && R0 && r && z && work, "fr_pmg_apply: null argument");
  CHECK(z != r && z != U && z != R0, "fr_pmg_apply: z aliases an input");
  CHECK(pmg_compatible(d, pc->mg), "fr_pmg_apply: pc has no matching coarse level (fr_pmg_factor)");
  CHECK(eps_mode == FR_EPS_ABS || eps_mode == FR_EPS_RMS, "fr_pmg_apply: bad eps_mode");
  CHECK(eps > 0.0, "fr_pmg_apply: eps must be positive");
  Carver cv(work);
  GmWork W = carve_gmres(cv, d, 1);
  ResArgs ra{};
  ra.U = U;
  ra.R0 = R0;
  ra.eps = eps;
  ra.eps_mode = eps_mode;
  ra.shift = shift;
  ra.nrm2 = W.scal;
  int np = 0;
  return pmg_apply(d, pc->d_factors, pc->precision, pc->mg, ra, r, nullptr, nullptr, z, W, W.partials + kPartZ, &np,
                   nullptr, S(s));
}

static fr_status check_step(const fr_disc* d, const fr_solver_opts* o, fr_step_stats* st, void* work) {
  CHECK(d && o && st && work, "step: null argument");
  fr_status c = check_gmres_opts(&o->lin);
  if (c != FR_OK) return c;
  CHECK(o->precond_precision == FR_F64 || o->precond_precision == FR_F32, "step: bad precond_precision");
  CHECK(o->lin.precond != FR_PC_PMG, "step: the time steps take element-Jacobi or LU-SGS (p-multigrid: "
                                     "fr_gmres_solve with fr_pmg_factor)");
  return FR_OK;
}

fr_status fr_row_step(const fr_disc* d, int scheme, double dt, double* U, const fr_solver_opts* o,
                      fr_step_stats* st, void* work, fr_stream s) {
  clear_error();
  fr_status c = check_step(d, o, st, work);
  if (c != FR_OK) return c;
  CHECK(U != nullptr && dt > 0.0, "fr_row_step: null state or dt <= 0");
  CHECK(row_scheme(scheme) != nullptr, "fr_row_step: scheme must be FR_ROW2/3/4");
  *st = fr_step_stats{};
  return row_step_impl(d, scheme, dt, U, *o, st, work, S(s));
}

fr_status fr_esdirk_step(const fr_disc* d, int scheme, double dt, double* U, const fr_solver_opts* o,
                         fr_step_stats* st, void* work, fr_stream s) {
  clear_error();
  fr_status c = check_step(d, o, st, work);
  if (c != FR_OK) return c;
  CHECK(U != nullptr && dt > 0.0, "fr_esdirk_step: null state or dt <= 0");
  CHECK(esdirk_scheme(scheme) != nullptr, "fr_esdirk_step: scheme must be FR_ESDIRK2/3/4");
  *st = fr_step_stats{};
  return esdirk_step_impl(d, scheme, dt, U, *o, st, work, S(s));
}

fr_status fr_bdf2_step(const fr_disc* d, double dt, const double* Unm1, const double* Un, double* Unp1,
                       const fr_solver_opts* o, fr_step_stats* st, void* work, fr_stream s) {
  clear_error();
  fr_status c = check_step(d, o, st, work);
  if (c != FR_OK) return c;
  CHECK(Un != nullptr && Unp1 != nullptr && dt > 0.0, "fr_bdf2_step: null state or dt <= 0");
  CHECK(Unp1 != Un && Unp1 != Unm1, "fr_bdf2_step: output aliases an input");
  *st = fr_step_stats{};
  return bdf2_step_impl(d, dt, Unm1, Un, Unp1, *o, st, work, S(s));
}

fr_status fr_wall_force(const fr_disc* d, const double* U, double* h_force, void* work, fr_stream s) {
  clear_error();
  CHECK(d && U && h_force && work, "fr_wall_force: null argument");
  CHECK(d->physics == FR_NS_BR1 && d->bc_south == FR_BC_WALL, "fr_wall_force: no wall on the eta = -1 side");
  double* part = (double*)work;
  FR_HIP(launch_ns_wall_flux(d, U, part, S(s)));
  std::vector<double> h(2 * (size_t)d->nx);
  FR_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, S(s)));
  FR_HIP(hipStreamSynchronize(S(s)));
  double fx = 0.0, fy = 0.0;
  for (int e = 0; e < d->nx; ++e) {
    fx += h[2 * e];
    fy += h[2 * e + 1];
  }
  h_force[0] = -fx;
  h_force[1] = -fy;
  return FR_OK;
}

fr_status fr_l2_error_vortex(const fr_disc* d, const double* U, int var, double t, const double* h_params,
                             double* h_err, void* work, fr_stream s) {
  clear_error();
  CHECK(d && U && h_params && h_err && work, "fr_l2_error_vortex: null argument");
  CHECK(var == 0 || var == 1, "fr_l2_error_vortex: var must be 0 (rho) or 1 (u)");
  Carver c(work);
  double* scal = (double*)c.take(256);
  double* partials = (double*)c.take(sizeof(double) * partials_count(d));
  FR_HIP(launch_l2_vortex(d, U, var, t, h_params, partials, scal, S(s)));
  double host[2];
  char* slot = (char*)d->h_pinned + 1024;
  FR_HIP(hipMemcpyAsync(slot, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, S(s)));
  FR_HIP(hipStreamSynchronize(S(s)));
  std::memcpy(host, slot, sizeof(host));
  *h_err = std::sqrt(host[0] / host[1]);
  return FR_OK;
}

size_t fr_mlp_weight_bytes(int n_in, int n_hidden, int n_out) {
  return mlp_weight_elems(n_in, n_hidden, n_out) * sizeof(uint16_t);
}
size_t fr_mlp_param_count(int n_in, int n_hidden, int n_out) { return mlp_param_elems(n_in, n_hidden, n_out); }
size_t fr_mlp_work_bytes(const fr_disc* d, int n_hidden, int batch) {
  if (d == nullptr) return 0;
  const int In = 16 * d->np, Out = 4 * d->np;
  return std::max(mlp_infer_bytes(d->nel, In, n_hidden, Out), mlp_train_bytes(std::max(batch, 1), In, n_hidden, Out));
}

static fr_status check_mlp(const fr_disc* d, const fr_mlp* net) {
  CHECK(net && net->d_w && net->d_b && net->d_norm, "null network buffers");
  CHECK(net->n_hidden >= 16 && net->n_hidden <= 4096, "n_hidden must be in 16..4096");
  if (d != nullptr) CHECK(net->n_in == 16 * d->np && net->n_out == 4 * d->np, "network sizes do not match the disc");
  return FR_OK;
}

fr_status fr_mlp_infer(const fr_disc* d, const fr_mlp* net, const double* U, const double* R, const double* Y1,
                       const double* Y2, double dt, double* x0, void* work, fr_stream s) {
  clear_error();
  CHECK(d && U && R && x0 && work && dt > 0.0, "fr_mlp_infer: null argument or dt <= 0");
  fr_status c = check_mlp(d, net);
  if (c != FR_OK) return c;
  FR_HIP(mlp_infer(d, net, U, R, Y1, Y2, dt, x0, work, S(s)));
  return FR_OK;
}

fr_status fr_mlp_forward(const fr_mlp* net, const uint16_t* x, int batch, float* y, void* work, fr_stream s) {
  clear_error();
  CHECK(x && y && work && batch > 0, "fr_mlp_forward: null argument or empty batch");
  fr_status c = check_mlp(nullptr, net);
  if (c != FR_OK) return c;
  char* p = (char*)work;
  uint16_t* H1 = (uint16_t*)p;
  uint16_t* H2 = (uint16_t*)(p + (((size_t)batch * net->n_hidden * 2 + 255) / 256) * 256);
  FR_HIP(mlp_forward(net, x, batch, y, H1, H2, S(s)));
  return FR_OK;
}

fr_status fr_mlp_fit_stats(const fr_disc* d, const fr_stage_log* log, fr_mlp* net, fr_stream s) {
  clear_error();
  CHECK(d && log && log->d_samples && log->count > 0, "fr_mlp_fit_stats: empty log");
  fr_status c = check_mlp(d, net);
  if (c != FR_OK) return c;
  FR_HIP(mlp_stats(log->d_samples, log->count, d->np, net->d_norm, S(s)));
  return FR_OK;
}

fr_status fr_mlp_sync(fr_mlp_trainer* tr, fr_stream s) {
  clear_error();
  CHECK(tr && tr->d_master, "fr_mlp_sync: null argument");
  fr_status c = check_mlp(nullptr, &tr->net);
  if (c != FR_OK) return c;
  FR_HIP(mlp_sync_weights(tr, S(s)));
  return FR_OK;
}

fr_status fr_mlp_train_step(const fr_disc* d, fr_mlp_trainer* tr, const fr_stage_log* log, const int* idx, int batch,
                            double* h_loss, void* work, fr_stream s) {
  clear_error();
  CHECK(d && tr && log && log->d_samples && idx && work && batch > 0, "fr_mlp_train_step: null argument");
  CHECK(tr->d_master && tr->d_grad && tr->d_m && tr->d_v, "fr_mlp_train_step: null trainer buffers");
  fr_status c = check_mlp(d, &tr->net);
  if (c != FR_OK) return c;
  const float* raw = log->d_samples;
  void* w = work;
  int np = 0;
  FR_HIP(mlp_train_group(&tr, &raw, &idx, 1, batch, d->np, &w, &np, S(s)));
  if (h_loss == nullptr) return FR_OK;  // asynchronous: no loss read-back
  FR_HIP(mlp_group_loss(&w, 1, batch, tr->net.n_in, tr->net.n_hidden, tr->net.n_out, np, h_loss, S(s)));
  return FR_OK;
}

size_t fr_mlp_group_work_bytes(const fr_disc* d, int n_hidden, int batch, int count) {
  if (d == nullptr || batch < 1 || count < 1 || count > kMlpGroupMax) return 0;
  return (size_t)count * mlp_train_bytes(batch, 16 * d->np, n_hidden, 4 * d->np);
}

fr_status fr_mlp_train_group(const fr_disc* d, fr_mlp_trainer* trs, const fr_stage_log* logs, int count,
                             const int* idx, int steps, int batch, const float* h_lr, double* h_loss, void* work,
                             fr_stream s) {
  clear_error();
  CHECK(d && trs && logs && idx && work, "fr_mlp_train_group: null argument");
  CHECK(batch > 0 && steps > 0, "fr_mlp_train_group: empty batch or no steps");
  CHECK(count >= 1 && count <= kMlpGroupMax, "fr_mlp_train_group: count must be in 1..8");
  for (int q = 0; q < count; ++q) {
    CHECK(trs[q].d_master && trs[q].d_grad && trs[q].d_m && trs[q].d_v, "fr_mlp_train_group: null trainer buffers");
    fr_status c = check_mlp(d, &trs[q].net);
    if (c != FR_OK) return c;
    CHECK(trs[q].net.n_hidden == trs[0].net.n_hidden, "fr_mlp_train_group: networks of different sizes");
    CHECK(logs[q].d_samples && logs[q].count > 0, "fr_mlp_train_group: empty log");
  }
  const int In = trs[0].net.n_in, H = trs[0].net.n_hidden, Out = trs[0].net.n_out;
  const size_t tb = mlp_train_bytes(batch, In, H, Out);
  fr_mlp_trainer* tp[kMlpGroupMax];
  const float* raws[kMlpGroupMax];
  const int* ip[kMlpGroupMax];
  void* works[kMlpGroupMax];
  for (int q = 0; q < count; ++q) {
    tp[q] = &trs[q];
    raws[q] = logs[q].d_samples;
    works[q] = (char*)work + (size_t)q * tb;
  }
  int np = 0;
  for (int k = 0; k < steps; ++k) {
    for (int q = 0; q < count; ++q) {
      ip[q] = idx + ((size_t)q * steps + k) * batch;
      if (h_lr != nullptr) trs[q].lr = h_lr[k];
    }
    FR_HIP(mlp_train_group(tp, raws, ip, count, batch, d->np, works, &np, S(s)));
  }
  if (h_loss != nullptr) FR_HIP(mlp_group_loss(works, count, batch, In, H, Out, np, h_loss, S(s)));
  return FR_OK;
}

// ---------------------------------------------------------------- 3D hexahedral FR
struct Work3 {
  void* traces;
  double* scal;
  double* partials;
  double* R;
  double* U1;
};
static size_t r256(size_t b) { return (b + 255) & ~(size_t)255; }
static Work3 carve3(const fr3d_disc* d, void* work) {
  char* p = (char*)work;
  Work3 w;
  w.traces = p;
  p += r256(fr3d_trace_bytes(d));
  w.scal = (double*)p;
  p += 256;
  w.partials = (double*)p;
  p += r256(sizeof(double) * std::max<size_t>(kRedBlocks, 5 * (size_t)d->nel));
  w.R = (double*)p;
  p += r256(sizeof(double) * d->ndof);
  w.U1 = (double*)p;
  return w;
}

fr_status fr3d_create(const fr3d_desc* desc, fr3d_disc** out) {
  clear_error();
  CHECK(desc != nullptr && out != nullptr, "fr3d_create: null argument");
  CHECK(desc->p >= 2 && desc->p <= 4, "fr3d_create: p must be 2 .. 4");
  CHECK(desc->nx >= 2 && desc->ny >= 2 && desc->nz >= 2, "fr3d_create: nx, ny and nz must be >= 2");
  CHECK((size_t)desc->nx * desc->ny * desc->nz < (1u << 28), "fr3d_create: mesh too large");
  CHECK(desc->flux == FR_RUSANOV || desc->flux == FR_ROE, "fr3d_create: bad flux");
  CHECK(desc->len[0] > 0.0 && desc->len[1] > 0.0 && desc->len[2] > 0.0, "fr3d_create: box lengths must be positive");
  CHECK(desc->gamma > 1.0 && desc->rgas > 0.0 && desc->mu >= 0.0 && desc->prandtl > 0.0,
        "fr3d_create: gamma > 1, R > 0, mu >= 0 and Pr > 0 required");
  fr3d_disc* d = new fr3d_disc{};
  d->nx = desc->nx;
  d->ny = desc->ny;
  d->nz = desc->nz;
  d->p = desc->p;
  d->n = desc->p + 1;
  d->np = d->n * d->n * d->n;
  d->nel = desc->nx * desc->ny * desc->nz;
  d->flux = desc->flux;
  d->ndof = (size_t)5 * d->nel * d->np;
  const int ne[3] = {desc->nx, desc->ny, desc->nz};
  for (int i = 0; i < 3; ++i) {
    d->lo[i] = desc->lo[i];
    d->h[i] = desc->len[i] / ne[i];
  }
  d->gamma = desc->gamma;
  d->rgas = desc->rgas;
  d->mu = desc->mu;
  d->prandtl = desc->prandtl;
  d->basis = make_basis(desc->p);
  *out = d;
  return FR_OK;
}

void fr3d_destroy(fr3d_disc* d) { delete d; }

size_t fr3d_ndof(const fr3d_disc* d) { return d ? d->ndof : 0; }

size_t fr3d_workspace_bytes(const fr3d_disc* d) {
  if (d == nullptr) return 0;
  return r256(fr3d_trace_bytes(d)) + 256 + r256(sizeof(double) * std::max<size_t>(kRedBlocks, 5 * (size_t)d->nel)) +
         2 * r256(sizeof(double) * d->ndof);
}

fr_status fr3d_solution_points(const fr3d_disc* d, double* xyz) {
  clear_error();
  CHECK(d && xyz, "fr3d_solution_points: null argument");
  const int n = d->n;
  const size_t per = (size_t)d->nel * d->np;
  for (int e = 0; e < d->nel; ++e) {
    const int ex = e % d->nx, ey = (e / d->nx) % d->ny, ez = e / (d->nx * d->ny);
    for (int k = 0; k < d->np; ++k) {
      const int a = k % n, b = (k / n) % n, c = k / (n * n);
      const size_t i = (size_t)e * d->np + k;
      xyz[i] = d->lo[0] + d->h[0] * (ex + 0.5 * (d->basis.x[a] + 1.0));
      xyz[per + i] = d->lo[1] + d->h[1] * (ey + 0.5 * (d->basis.x[b] + 1.0));
      xyz[2 * per + i] = d->lo[2] + d->h[2] * (ez + 0.5 * (d->basis.x[c] + 1.0));
    }
  }
  return FR_OK;
}

fr_status fr3d_residual(const fr3d_disc* d, const double* U, double* R, void* work, fr_stream s) {
  clear_error();
  CHECK(d && U && R && work, "fr3d_residual: null argument");
  CHECK(U != R, "fr3d_residual: U and R alias");
  FR_HIP(launch_fr3d_residual(d, 0, U, nullptr, nullptr, 0.0, 0.0, FR_EPS_ABS, nullptr, R, work, S(s)));
  return FR_OK;
}

fr_status fr3d_jf_matvec(const fr3d_disc* d, const double* U, const double* R0, const double* v, double shift,
                         double eps, int eps_mode, double* w, void* work, fr_stream s) {
  clear_error();
  CHECK(d && U && R0 && v && w && work, "fr3d_jf_matvec: null argument");
  CHECK(w != U && w != R0 && w != v, "fr3d_jf_matvec: the output aliases an input");
  CHECK(eps_mode == FR_EPS_ABS || eps_mode == FR_EPS_RMS, "fr3d_jf_matvec: bad eps_mode");
  CHECK(eps > 0.0, "fr3d_jf_matvec: eps must be positive");
  Work3 k = carve3(d, work);
  if (eps_mode == FR_EPS_RMS) FR_HIP(launch_norm2(v, d->ndof, k.partials, k.scal, nullptr, S(s)));
  FR_HIP(launch_fr3d_residual(d, 1, U, v, R0, shift, eps, eps_mode, k.scal, w, k.traces, S(s)));
  return FR_OK;
}

fr_status fr3d_ssprk3_step(const fr3d_disc* d, double* U, double dt, void* work, fr_stream s) {
  clear_error();
  CHECK(d && U && work, "fr3d_ssprk3_step: null argument");
  CHECK(dt > 0.0, "fr3d_ssprk3_step: dt must be positive");
  Work3 k = carve3(d, work);
  const size_t n = d->ndof;
  FR_HIP(launch_fr3d_residual(d, 0, U, nullptr, nullptr, 0.0, 0.0, FR_EPS_ABS, nullptr, k.R, k.traces, S(s)));
  FR_HIP(launch_fr3d_combine(k.U1, U, U, k.R, 0.0, 1.0, dt, n, S(s)));          // U1 = U + dt R(U)
  FR_HIP(launch_fr3d_residual(d, 0, k.U1, nullptr, nullptr, 0.0, 0.0, FR_EPS_ABS, nullptr, k.R, k.traces, S(s)));
  FR_HIP(launch_fr3d_combine(k.U1, U, k.U1, k.R, 0.75, 0.25, dt, n, S(s)));     // U2 = 3/4 U + 1/4 (U1 + dt R(U1))
  FR_HIP(launch_fr3d_residual(d, 0, k.U1, nullptr, nullptr, 0.0, 0.0, FR_EPS_ABS, nullptr, k.R, k.traces, S(s)));
  FR_HIP(launch_fr3d_combine(U, U, k.U1, k.R, 1.0 / 3.0, 2.0 / 3.0, dt, n, S(s)));  // U = 1/3 U + 2/3 (U2 + dt R(U2))
  return FR_OK;
}

fr_status fr3d_dissipation(const fr3d_disc* d, const double* U, double rho0, double* h_out, void* work, fr_stream s) {
  clear_error();
  CHECK(d && U && h_out && work && rho0 > 0.0, "fr3d_dissipation: null argument or rho0 <= 0");
  Work3 k = carve3(d, work);
  FR_HIP(launch_fr3d_dissipation(d, U, k.partials, S(s)));
  FR_HIP(launch_finalize(k.partials, d->nel, 5, 5, k.scal, nullptr, S(s)));
  double h[5];  // int rho|u|^2/2, int S^d:S^d, int p div u, int p, int div u
  FR_HIP(hipMemcpyAsync(h, k.scal, sizeof(h), hipMemcpyDeviceToHost, S(s)));
  FR_HIP(hipStreamSynchronize(S(s)));
  const double V = d->h[0] * d->h[1] * d->h[2] * d->nel;
  h_out[0] = h[0] / (rho0 * V);
  h_out[1] = 2.0 * d->mu * h[1] / (rho0 * V);
  // int (p - <p>) div u = int p div u - <p> int div u (see the declaration)
  h_out[2] = -(h[2] - (h[3] / V) * h[4]) / (rho0 * V);
  return FR_OK;
}

size_t fr3d_ejacobi_bytes(const fr3d_disc* d) { return d ? fr3d_block_bytes(d) : 0; }

size_t fr3d_step_workspace_bytes(const fr3d_disc* d, int m) {
  if (d == nullptr || m < 1 || m > kMaxM) return 0;
  return fr3d_step_bytes(d, m);
}

fr_status fr3d_ejacobi_assemble(const fr3d_disc* d, const double* U, double shift, double* blocks, void* work,
                                fr_stream s) {
  clear_error();
  CHECK(d && U && blocks && work, "fr3d_ejacobi_assemble: null argument");
  return fr3d_assemble_impl(d, U, shift, blocks, work, S(s));
}

fr_status fr3d_ejacobi_factor(const fr3d_disc* d, const double* U, double shift, double* inv, void* work,
                              fr_stream s) {
  clear_error();
  CHECK(d && U && inv && work, "fr3d_ejacobi_factor: null argument");
  return fr3d_factor_impl(d, U, shift, inv, work, S(s));
}

fr_status fr3d_ejacobi_apply(const fr3d_disc* d, const double* inv, const double* r, double* z, fr_stream s) {
  clear_error();
  CHECK(d && inv && r && z, "fr3d_ejacobi_apply: null argument");
  CHECK(r != z, "fr3d_ejacobi_apply: r and z alias");
  return fr3d_apply_impl(d, inv, r, z, S(s));
}

fr_status fr3d_gmres_solve(const fr3d_disc* d, const double* inv, const double* U, const double* R0, double shift,
                           const double* b, double* x, const fr_gmres_opts* o, fr_gmres_stats* st, void* work,
                           fr_stream s) {
  clear_error();
  CHECK(d && inv && U && R0 && b && x && o && st && work, "fr3d_gmres_solve: null argument");
  CHECK(x != b && x != U && x != R0, "fr3d_gmres_solve: x aliases an input");
  CHECK(o->rtol > 0.0, "fr3d_gmres_solve: rtol must be positive");
  *st = fr_gmres_stats{};
  return fr3d_gmres_impl(d, inv, U, R0, shift, b, x, *o, st, work, S(s));
}

static fr_status check3_step(const fr3d_disc* d, const void* U, double dt, const fr_solver_opts* o,
                             fr_step_stats* st, void* work, const char* who) {
  if (!(d && U && o && st && work)) return set_error(FR_EINVAL, std::string(who) + ": null argument");
  if (!(dt > 0.0)) return set_error(FR_EINVAL, std::string(who) + ": dt must be positive");
  if (!(o->lin.rtol > 0.0)) return set_error(FR_EINVAL, std::string(who) + ": lin.rtol must be positive");
  *st = fr_step_stats{};
  return FR_OK;
}

fr_status fr3d_row_step(const fr3d_disc* d, int scheme, double dt, double* U, const fr_solver_opts* o,
                        fr_step_stats* st, void* work, fr_stream s) {
  clear_error();
  fr_status c = check3_step(d, U, dt, o, st, work, "fr3d_row_step");
  if (c != FR_OK) return c;
  return fr3d_row_impl(d, scheme, dt, U, *o, st, work, S(s));
}

fr_status fr3d_esdirk_step(const fr3d_disc* d, int scheme, double dt, double* U, const fr_solver_opts* o,
                           fr_step_stats* st, void* work, fr_stream s) {
  clear_error();
  fr_status c = check3_step(d, U, dt, o, st, work, "fr3d_esdirk_step");
  if (c != FR_OK) return c;
  return fr3d_esdirk_impl(d, scheme, dt, U, *o, st, work, S(s));
}

fr_status fr3d_bdf2_step(const fr3d_disc* d, double dt, const double* Unm1, const double* Un, double* Unp1,
                         const fr_solver_opts* o, fr_step_stats* st, void* work, fr_stream s) {
  clear_error();
  fr_status c = check3_step(d, Un, dt, o, st, work, "fr3d_bdf2_step");
  if (c != FR_OK) return c;
  CHECK(Unp1 != nullptr && Unp1 != Un && Unp1 != Unm1, "fr3d_bdf2_step: Unp1 null or aliasing an input");
  return fr3d_bdf2_impl(d, dt, Unm1, Un, Unp1, *o, st, work, S(s));
}

int fr_scheme_table(int kind, int scheme, double* a, double* c, double* b, double* gamma) {
  if (!a || !b || !gamma) return FR_EINVAL;
  if (kind == 0) {
    const RowScheme* r = row_scheme(scheme);
    if (!r || !c) return FR_EINVAL;
    for (int i = 0; i < r->s; ++i) {
      for (int j = 0; j < r->s; ++j) {
        a[i * r->s + j] = r->a[i][j];
        c[i * r->s + j] = r->c[i][j];
      }
      b[i] = r->m[i];
    }
    *gamma = r->gamma;
    return r->s;
  }
  if (kind == 1) {
    const EsdirkScheme* e = esdirk_scheme(scheme);
    if (!e) return FR_EINVAL;
    for (int i = 0; i < e->s; ++i) {
      for (int j = 0; j < e->s; ++j) a[i * e->s + j] = e->a[i][j];
      b[i] = e->b[i];
    }
    *gamma = e->gamma;
    return e->s;
  }
  return FR_EINVAL;
}

}  // extern "C"
