// Internal declarations of the frjf library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/frjf.h"

namespace frjf {

constexpr int kMaxN = 7;  // P <= 6

// 1D reference-element tables of degree P, passed to kernels by value.
struct Basis {
  int n;                   // P + 1
  double x[kMaxN];         // Gauss-Legendre points
  double w[kMaxN];         // Gauss weights
  double D[kMaxN][kMaxN];  // D[a][b] = l_b'(x_a)
  double lm[kMaxN];        // l_b(-1)
  double lp[kMaxN];        // l_b(+1)
  double gL[kMaxN];        // g_L'(x_a), left Radau correction derivative
  double gR[kMaxN];        // g_R'(x_a), right Radau correction derivative
  double kLL, kLR, kRL, kRR;  // sum_a l_a(s) g_t'(x_a): trace of a lifted face jump (BR1)
};

Basis make_basis(int P);

struct Phys {
  double gamma, rgas, mu, prandtl;
  double cp_over_pr;  // kappa / mu = Cp / Pr
};

}  // namespace frjf

struct fr_disc {
  int nx, ny, p, n, np, nb, nel;
  int physics, flux;
  int visc, bc_south, bc_north;  // Navier-Stokes: FR_BR1 / FR_BR2, FR_BC_* of the eta-sides
  double qfar[4];                // far-field state
  size_t ndof;
  frjf::Phys phys;
  frjf::Basis basis;
  const double* nodes;
  int device;
  int ncu;  // compute units of the device (persistent-grid sizing)
  // pinned, mapped host scratch: [0, 1 KiB) GMRES status written by the device,
  // [1 KiB, 4 KiB) staging of synchronous device-to-host reads
  void* h_pinned;
  void* d_pinned;  // device-side address of h_pinned
  // device address of the library's static scratch array on this disc's device (looked
  // up once per device by fr_disc_create; used by fr_jf_matvec_noalloc)
  void* d_scratch;
  hipEvent_t ev[4];
};

// 3D hexahedral discretisation (uniform elements of a triply periodic box)
struct fr3d_disc {
  int nx, ny, nz, p, n, np, nel, flux;
  size_t ndof;
  double lo[3], h[3];
  double gamma, rgas, mu, prandtl;
  frjf::Basis basis;
};

namespace frjf {

// error reporting (thread-local message)
fr_status set_error(fr_status st, const std::string& msg);
void clear_error();

#define FR_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return ::frjf::set_error(FR_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------- launchers
// Residual family.  mode 0: out = R(U);  mode 1: out = shift v - (R(U + e v) - R0)/e;
// mode 2: out = b - [shift v - (R(U + e v) - R0)/e].  e from *nrm2 (rms) or eps (abs).
struct ResArgs {
  const double* U;
  const double* V;
  const double* R0;
  const double* B;
  double* out;
  double* nrm2;         // device scalar ||v||^2 (rms mode)
  // optional, rms mode: nrm2_nb partial sums of ||v||^2 in place of a finished *nrm2;
  // small meshes add them inside the residual kernel, otherwise the launcher first
  // sums them into *nrm2
  const double* nrm2_part;
  int nrm2_nb;
  const int* skip;      // optional device flag: nonzero -> kernel returns at once
  double eps;
  int eps_mode;
  double shift;
  double* grad;         // BR1 face-gradient traces (workspace)
  // optional, JF product on small Euler meshes (see residual_dots_blocks): the first
  // DCGS2 pass over the product's output w, dnv <= kJfDotsMax basis vectors at dV:
  // per-workgroup partial sums of <V_t, w>, <V_t, V_{dnv-1}> and <w, w> in the row
  // layout of launch_dcgs2_dots, into dpart
  const double* dV;
  int dnv;
  double* dpart;
  // optional, b - A x on small Euler meshes (residual_dots_blocks > 0): per-tile partial
  // sums of ||b - A x||^2 into opart
  double* opart;
};
hipError_t launch_residual(const fr_disc* d, int mode, const ResArgs& a, hipStream_t s);
// Workgroups of the JF product when it can also run the first DCGS2 pass (small Euler
// meshes, at most kRedBlocks tiles, up to kJfDotsMax basis vectors), else 0.
constexpr int kJfDotsMax = 20;
int residual_dots_blocks(const fr_disc* d);

// Vector operations (flat arrays of n doubles).
// Sum of squares with a deterministic two-level reduction; result in *out (device).
hipError_t launch_norm2(const double* x, size_t n, double* partials, double* out,
                        const int* skip, hipStream_t s);
// Partial sums of ||x||^2 only: *nb <= kRedBlocks of them into partials.
hipError_t launch_norm2_parts(const double* x, size_t n, double* partials, int* nb, const int* skip, hipStream_t s);
// y = sum_i c[i] * x[i] (k <= 8); pointers and coefficients passed by value
hipError_t launch_lincomb(double* y, int k, const double* const* x, const double* c, size_t n,
                          hipStream_t s);

// element-Jacobi
// grad: BR1 gradient-trace workspace (Navier-Stokes only, else unused)
hipError_t launch_ejacobi_assemble(const fr_disc* d, const double* U, double shift, void* out,
                                   int precision, int invert, double* grad, hipStream_t s);
// In-place inversion of nblk FP64 blocks of order 100, column-major (other orders: hipErrorInvalidValue).
hipError_t launch_gj_rows_f64(int nb, double* blocks, int nblk, hipStream_t s);
// In-place inversion of nblk FP32 blocks of order nb (36, 64 or 100), column-major, on MFMA.
hipError_t launch_gj_mfma_f32(int nb, float* blocks, int nblk, hipStream_t s);
// In-place inversion of nblk blocks of order 144 or 196 (P = 5, 6), column-major, the rows
// split over column segments held in registers (gj_wide.hip).
hipError_t launch_gj_wide_f64(int nb, double* blocks, int nblk, hipStream_t s);
hipError_t launch_gj_wide_f32(int nb, float* blocks, int nblk, hipStream_t s);
// FP32 inversion of any supported order: MFMA for 36, 64, 100, segmented rows for 144, 196.
hipError_t launch_invert_f32(int nb, float* blocks, int nblk, hipStream_t s);
// In-place inversion of nblk FP64 blocks of order nb: on MFMA (k_gj_mfma) for 36 and 64,
// by k_gj_rows for 100.
hipError_t launch_invert_f64(int nb, double* blocks, int nblk, hipStream_t s);
hipError_t launch_ejacobi_invert_blocks(const fr_disc* d, const double* blocks, void* out,
                                        int precision, hipStream_t s);
struct GivensIn;
// z = M^{-1} r, or with gv: the Givens update of step gv->st->j, then
// z = M^{-1} (r / ||r||) with r_store receiving r / ||r|| (||r||^2 from gv's partials).
// Partial sums of ||z||^2 go to partials when nrm2 (then summed into *nrm2) or nparts
// (then only their count is returned, for a consumer that adds them itself) is given.
// One pass of the LU-SGS preconditioner (PASS 1, 2, 3; see ejacobi.hip) over the
// element-Jacobi inverse blocks; even nx and ny only.  Partial sums of ||out||^2 (PASS 2:
// ||out2||^2) go to partials, their count to *nparts.
hipError_t launch_lusgs_pass(const fr_disc* d, const void* factors, int precision, int pass, const double* r,
                             const double* w, const double* y, double* out, double* out2, const GivensIn* gv,
                             double* r_store, double* partials, int* nparts, const int* skip, hipStream_t s);
hipError_t launch_ejacobi_solve(const fr_disc* d, const void* factors, int precision,
                                const double* r, const GivensIn* gv, double* r_store,
                                double* z, double* partials, int* nparts, double* nrm2,
                                const int* skip, hipStream_t s);

hipError_t launch_solution_points(const fr_disc* d, double* xy, hipStream_t s);
// force of the fluid on the wall (ns.hip): per element of row 0, its wall face's momentum flux
hipError_t launch_ns_wall_flux(const fr_disc* d, const double* U, double* part, hipStream_t s);
// 3D hexahedral FR (fr3d.hip)
size_t fr3d_trace_bytes(const fr3d_disc* d);
hipError_t launch_fr3d_residual(const fr3d_disc* d, int mode, const double* U, const double* V, const double* R0,
                                double shift, double eps, int eps_mode, const double* nrm2, double* out, void* work,
                                hipStream_t s);
hipError_t launch_fr3d_residual_subset(const fr3d_disc* d, const double* U, double* out, void* work,
                                       const int* elist, int count, int copies, size_t face_stride,
                                       bool faces_only, hipStream_t s);
hipError_t launch_fr3d_combine(double* out, const double* A, const double* Bv, const double* R, double alpha,
                               double beta, double dt, size_t n, hipStream_t s);
hipError_t launch_fr3d_dissipation(const fr3d_disc* d, const double* U, double* part, hipStream_t s);
hipError_t launch_l2_vortex(const fr_disc* d, const double* U, int var, double t, const double* prm,
                            double* partials, double* out, hipStream_t s);

// State vectors of a time step's workspace (stage vectors, PTC state, increments).
constexpr int kStepVecs = 15;
constexpr int kRedBlocks = 1024;  // blocks of the grid-stride vector kernels
constexpr int kRedThreads = 256;

// Arnoldi (CGS2) device state, one per GMRES solve, in the workspace.
constexpr int kMaxM = 64;
struct GmState {
  double H[(kMaxM + 1) * kMaxM];  // column-major: H[j*(M+1) + i]
  double cs[kMaxM], sn[kMaxM];
  double g[kMaxM + 1];
  double h1[kMaxM + 1];
  double h2[kMaxM + 1];
  double y[kMaxM];
  double target;       // rtol * r_ref
  double hn;           // ||w|| after orthogonalisation
  double w0;           // ||w|| before
  // status block copied to the host after every Arnoldi step
  double rest;         // |g_{j+1}|, the least-squares residual
  double beta;
  int j;               // Arnoldi steps done in this cycle
  int stop;            // 1: converged / breakdown / nan -> the rest of the cycle is skipped
  int why;             // 1 converged, 2 breakdown, 3 nan
  int evals;           // JF products of the cycle that ran (counted by the DCGS2 second pass)
  int done;            // converged or NaN: the cycle's closing kernels for a restart return at once
  struct GmStatus* hslot;  // mapped host memory receiving the status after every step
  // restart decisions on the device, so the host enqueues the next cycle without waiting
  struct Final {
    int fin;             // the solve has ended: its later kernels return at once
    int result;          // its fr_status once fin
    int iters, evals, restarts;
    int steps;           // Arnoldi steps that ran (one preconditioner application each)
    double r_final;      // least-squares or true residual norm
    double r_ref;        // the norm the tolerance is relative to
  } fz;
};
struct GmStatus {
  double rest, beta;
  int j, stop, why, evals;
};
// V: nv vectors of n doubles stored back to back (vector i at V + i*n).
// Partial sums of the Arnoldi step, stored value-major (value t of workgroup b at
// t kRedBlocks + b): the CGS2 passes use partials[0 ..) and partials[kPartSecond ..)
// (32 values each), the DCGS2 first pass partials[0 ..) (up to 64 values) and its
// second pass partials[2 kPartSecond ..); rows of the chunked dot kernel for long
// restarts are kPartStride apart.
constexpr int kPartStride = kMaxM + 2;
constexpr size_t kPartSecond = (size_t)kRedBlocks * 32;
// Offset of the DCGS2 second pass's partial sums of ||w'||^2 (the first pass, alone or
// fused into the JF product, fills up to 2 x 32 rows before it).
constexpr size_t kDcgsNormOff = 2 * kPartSecond;
// Offset of the preconditioner application's partial sums of ||z_j||^2 inside an
// Arnoldi step.  The JF product that reads them may also write the first DCGS2 pass's
// rows (up to 2 kJfDotsMax of them) while other tiles still read, so this slot lies
// past every row of both passes.
constexpr size_t kPartZ = kDcgsNormOff + kRedBlocks;
static_assert(2 * (size_t)kJfDotsMax * kRedBlocks <= kPartZ, "fused DCGS2 rows overlap the ||z||^2 partials");
static_assert(2 * kPartSecond <= kPartZ, "DCGS2 first-pass rows overlap the ||z||^2 partials");
static_assert(kPartZ + kRedBlocks <= (size_t)kRedBlocks * (kMaxM + 2), "||z||^2 partials past the workspace");
// Workgroups of the CGS passes over n entries (<= kRedBlocks), i.e. the number of partial
// sums of ||w||^2 that the last pass leaves.
int cgs_blocks(size_t n);
// One Arnoldi orthogonalisation by CGS2: h1 = V^T w, w -= V h1, h2 = V^T w,
// w -= V h2, partial sums of ||w||^2; h1 and h2 go to st.  partials: at least
// 2 kPartSecond doubles.
hipError_t launch_arnoldi_cgs2(const double* V, int nv, double* w, double* partials, GmState* st, int M, size_t n,
                               hipStream_t s);
// The Givens update of Arnoldi step st->j from the nb partial sums of ||w||^2.
hipError_t launch_givens(GmState* st, const double* norm_part, int nb, int M, hipStream_t s);
// DCGS2 (restarts up to 32): one Arnoldi orthogonalisation in two passes over V, the
// re-orthogonalisation of basis vector nv-1 delayed to this step; finishes column nv-2
// of the Hessenberg matrix.  partials: at least 2 kPartSecond + kRedBlocks doubles.
bool dcgs2_supported(int m);
hipError_t launch_arnoldi_dcgs2(double* V, int nv, double* w, double* partials, GmState* st, int M, size_t n,
                                hipStream_t s);
// Where the second pass leaves its partial sums of ||w'||^2 (cgs_blocks(n) of them).
const double* dcgs2_norm_partials(const double* partials);
// The cycle's last column (first pass) rotated with ||w'|| from those partials.
hipError_t launch_dcgs2_last(GmState* st, const double* partials, int nb, int M, hipStream_t s);
// The second DCGS2 pass alone, its first pass's partial rows from nb1 workgroups of
// another kernel (the JF product).
hipError_t launch_dcgs2_update(double* V, int nv, double* w, double* partials, int nb1, GmState* st, int M,
                               size_t n, hipStream_t s);
// Run by the preconditioner kernel that starts the next Arnoldi step, which scales w by
// 1/||w|| (||w||^2 from norm_part): CGS2: the Givens update of the previous step;
// DCGS2 (lagged): ||w|| stored as the first-pass h_{j+1,j}, and on breakdown or NaN
// the first-pass column rotated as it stands.
struct GivensIn {
  GmState* st;
  const double* norm_part;  // nb <= kRedBlocks partial sums of ||w||^2
  int nb, M;
  int lagged;
};
// Cycle start: beta = sqrt(*beta2), v0 = r / beta, the cycle state reset (hslot); first:
// the solve's reference norm (ref, or beta for ref <= 0), target rtol * r_ref and totals,
// and an end before any step for a non-finite or converged beta; a later cycle does
// nothing once the solve has ended.
hipError_t launch_gm_start(GmState* st, const double* beta2, double rtol, double ref, int M, GmStatus* hslot,
                           double* v0, const double* r, size_t n, int first, hipStream_t s);
// End of a restart cycle (after the true residual's ||r||^2 in *beta2): the totals, and
// the decision to end the solve (converged, NaN, breakdown, max_iters) or restart.
hipError_t launch_gm_cycle_end(GmState* st, const double* beta2, int max_iters, int dcgs, hipStream_t s);
// The same with ||r||^2 from nbo <= kRedBlocks partial sums (stored to *beta2 as well).
hipError_t launch_gm_cycle_end_parts(GmState* st, double* beta2, const double* opart, int nbo, int max_iters,
                                     int dcgs, hipStream_t s);
// Sum partials[b*stride + i] over b < nblocks into out[i], i < nv (one workgroup).
hipError_t launch_finalize(const double* partials, int nblocks, int stride, int nv, double* out, const int* skip,
                           hipStream_t s);
// Number of workgroups of the grid-stride reductions over n entries (<= kRedBlocks).
int red_blocks(size_t n);
// End of a cycle: y from the rotated Hessenberg matrix and x += Z y for the st->j
// columns (x unchanged after NaN or without columns), with partial sums of ||x||^2 in
// xpart (*nb_out of them, at most kRedBlocks; M bounds st->j).
hipError_t launch_gm_update_x(double* x, const double* Z, int M, const GmState* st, size_t n, double* xpart,
                              int* nb_out, hipStream_t s);

// learned warm start (mlp.hip)
size_t mlp_weight_elems(int In, int H, int Out);
size_t mlp_param_elems(int In, int H, int Out);
size_t mlp_infer_bytes(int nel, int In, int H, int Out);
size_t mlp_train_bytes(int B, int In, int H, int Out);
hipError_t mlp_forward(const fr_mlp* net, const uint16_t* X, int B, float* Y, uint16_t* H1, uint16_t* H2,
                       hipStream_t s);
hipError_t mlp_infer(const fr_disc* d, const fr_mlp* net, const double* U, const double* R, const double* Y1,
                     const double* Y2, double dt, double* x0, void* work, hipStream_t s);
hipError_t mlp_log(const fr_disc* d, fr_stage_log* log, const double* U, const double* R, const double* Y1,
                   const double* Y2, const double* Y, double dt, hipStream_t s);
hipError_t mlp_stats(const float* raw, int count, int Np, float* norm, hipStream_t s);
constexpr int kMlpGroupMax = 8;  // networks trained together (mlp_train_group)
hipError_t mlp_train_group(fr_mlp_trainer* const* trs, const float* const* raws, const int* const* idx, int count,
                           int B, int Np, void* const* works, int* nparts, hipStream_t s);
hipError_t mlp_group_loss(void* const* works, int count, int B, int In, int H, int Out, int nparts, double* h_loss,
                          hipStream_t s);
hipError_t mlp_sync_weights(fr_mlp_trainer* tr, hipStream_t s);


}  // namespace frjf
