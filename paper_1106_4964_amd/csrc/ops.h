// Internal host-side entry points of libovl (called by the C ABI in abi.hip
// and by the higher-level drivers: sign function, solvers, eigensolver).
#pragma once

#include "core.h"

namespace ovl {

// ---------------------------------------------------------------- stencil
// out = G( a*in + b*hop(in) ) + sum_j cv[j] * G_j(v[j])
//   hop(in)(x) = sum_mu [ U_mu(x)(1-gamma_mu) in(x+mu) + U_mu(x-mu)^dag (1+gamma_mu) in(x-mu) ]
//   G = gamma5 if g5 else 1;  G_j = gamma5 if bit j of g5v else 1.
// Output sites: parities [par0, par0 + npar).  A batch of nrhs vectors is
// vstride bytes apart (inputs, outputs and the extra vectors alike).
struct StencilArgs {
  Geo g;
  void* out;
  const void* in;
  const void* links;
  const void* v[3];
  double cv[3];
  int nv;
  int g5v;
  double a, b;
  int g5;
  int par0, npar;
  size_t vstride;
  // 1: consecutive blocks of a parity walk t at a fixed tile of the (x, y, z)
  // half-slice, so t-neighbours are reused from cache; Z >= 2: blocks walk t
  // over a slab of Z z-planes before the next slab; 0: blocks follow h
  int tmaj = 0;
};


void launch_stencil(const StencilArgs& A, int prec, int recon, int nrhs, hipStream_t s);
// Stencil shape selection: mode 1 autotunes (default), 0 uses the static
// default (largest KR <= 4, <= 2 for FP64, dividing nrhs; 256 threads).
// Changing the mode clears the tuned table.
void set_tune_mode(int mode);
// Tuned shape of a configuration, if any: returns 1 and fills kr, bs, pipe.
int stencil_shape(int prec, int recon, int nv, int nrhs, int npar, int nh, int* shape5);
// Pins the shape of a configuration (tests, measurements).
void force_shape(int prec, int recon, int nv, int nrhs, int npar, int nh, const int* shape5);

// Representation of the links that operators at spinor precision prec use.
const void* gauge_links(const ovl_gauge* u, int prec, int* recon);

// ------------------------------------------------------------------ BLAS1
// Vectors of `n16` 16-byte blocks each (a whole batch can be passed as one
// vector).  Scalars in device memory are FP64 complex (re, im).
void blas_axpy(int prec, size_t n16, const double* a, const void* x, void* y, int nrhs, size_t vstride,
               hipStream_t s);
void blas_xpay(int prec, size_t n16, const void* x, const double* a, void* y, int nrhs, size_t vstride,
               hipStream_t s);
// y = gamma5 x for a batch of nrhs vectors of vstride bytes each.
void blas_gamma5(int prec, size_t vstride, const void* x, void* y, int nrhs, hipStream_t s);
// In place: keep chirality dev_sector[r] (+1 or -1; 0 = unchanged) of vector r.
void blas_chiral(int prec, size_t vstride, void* x, int nrhs, const int* dev_sector, hipStream_t s);
void blas_convert(int sprec, const void* src, int dprec, void* dst, size_t nsites, int nrhs, hipStream_t s);
// y(py) = a x(px) + b y(py) for a batch of nrhs lattice vectors (nsites
// sites each); a, b: device arrays of one complex (re, im) per rhs; b may be
// null (y = a x, y not read).  Arithmetic in the wider of the two types.
void blas_axpby(int px, const void* x, const double* a, int py, void* y, const double* b, size_t nsites, int nrhs,
                hipStream_t s);
// y = 0 over `bytes` (a multiple of 16), as a kernel.
void blas_zero(void* y, size_t bytes, hipStream_t s);
// Deterministic two-stage reductions; results (re, im) per rhs written to
// device memory dev_out[2*rhs].
void blas_dot(int prec, size_t n16, const void* x, const void* y, int nrhs, size_t vstride, double* dev_out,
              hipStream_t s);
void blas_norm2(int prec, size_t n16, const void* x, int nrhs, size_t vstride, double* dev_out,
                hipStream_t s);

// ------------------------------------------------------- tall-skinny blocks
// V: ell FP64 basis vectors (library layout, back to back); psi, Y: batch of
// R <= 12 vectors at precision prec.  C, K: device arrays of ell*R complex,
// index i*R + r.
void block_dot(const ovl_geom* g, const void* V, int ell, const void* psi, int prec, int R, double2* C,
               hipStream_t s);
void block_axpy(const ovl_geom* g, const void* V, int ell, const double2* K, void* Y, int prec, int R, bool keep,
                hipStream_t s);
// In place: V[:, j] = sum_{i<K} V[:, i] S[i + K*j] for j < k (FP64 basis, S on the device, K <= 512).
void block_rotate_inplace(const ovl_geom* g, void* V, int K, const double2* S, int k, hipStream_t s);

// ------------------------------------------------------------ sign / overlap
void lowmode_project(const ovl_lowmodes* lm, const void* psi, void* psih, void* w, int prec, int nrhs, int g5w,
                     hipStream_t s);
// The same projection with no device allocation: its scratch (coefficients
// and split-K partials) lives in a static per-device array.  Calls that
// overlap on one GPU share that array and race.
void lowmode_project_static(const ovl_lowmodes* lm, const void* psi, void* psih, void* w, int prec, int nrhs,
                            hipStream_t s);
// mode 0: sign(H_w) in;  1: D(m) in;  2: D(m)^dag in
void overlap_apply(void* out, const void* in, const ovl_gauge* u, double rho, double m, const ovl_sign* sg,
                   const ovl_lowmodes* lm, int mode, int prec, int nrhs, hipStream_t s);
// out = ap in + am gamma5 sign(H_w) in  (the general combine behind D(m))
void overlap_combine(void* out, const void* in, const ovl_gauge* u, double rho, double ap, double am,
                     const ovl_sign* sg, const ovl_lowmodes* lm, int prec, int nrhs, hipStream_t s);
// out = ap in + am sign(H_w) gamma5 in
void overlap_combine_dag(void* out, const void* in, const ovl_gauge* u, double rho, double ap, double am,
                         const ovl_sign* sg, const ovl_lowmodes* lm, int prec, int nrhs, hipStream_t s);

// The low part of eq. 9 for a batch of R FP64 residuals:
// x += sum_i xi_i (xi_i^dag r) / (rho d_i + m (1 - d_i/2)),  r -= sum_i xi_i (xi_i^dag r).
void deflate(const ovl_deflation* df, double rho, double m, void* x, void* r, int R, hipStream_t s);

// Eigen-decomposition of a Hermitian n x n matrix (column-major) on the
// host: ascending eigenvalues w, eigenvectors V (column-major).
void host_heev(int n, std::vector<std::complex<double>> A, std::vector<double>& w,
               std::vector<std::complex<double>>& V);

int cg_solve(void* x, const void* b, int R, const ovl_gauge* u, double rho, double m, const ovl_sign* sg,
             const ovl_lowmodes* lm, double tol, int maxiter, const ovl_solve_opts* o, ovl_solve_stats* st,
             hipStream_t us);

// out = M in for one FP32 spinor (learned preconditioner).
void net_apply(const ovl_net* net, const ovl_gauge* u, const void* in, void* out, int nrhs, hipStream_t s);

// Counters of stencil work issued from the host (not counting graph replays).
void count_stencil(int nrhs);
// Launch timer: mode 1 clears and enables, 0 disables, 2 clears.
void stencil_timer(int mode);
void stencil_timer_read(int prec, int recon, int nv, int nrhs, int64_t* launches, double* ms);

}  // namespace ovl
