// Polynomial sign function with low-mode projection, and the overlap
// operator (arXiv:1106.4964 Sec. II eq. 3-8, Sec. V).
//
//   sign(H_w) psi = sum_i sign(lambda_i) (eta_i^dag psi) eta_i + Q P(Q^2) psi_h,
//   psi_h = psi - sum_i (eta_i^dag psi) eta_i,   Q = H_w / lam_max,
//   P(x) = sum_k c_k T_k(y),  y = (2x - 1 - eps)/(1 - eps),
// with P(Q^2) psi_h evaluated by the Clenshaw recursion
//   b_k = c_k psi_h + 2 Y b_{k+1} - b_{k+2},  P psi_h = c_0 psi_h + Y b_1 - b_2,
//   Y = (2 Q^2 - 1 - eps)/(1 - eps),
// each step being two stencil launches: t = H_w b_{k+1}, then
//   b_k = s H_w t + c1 b_{k+1} - b_{k+2} + c_k psi_h      (one fused epilogue)
// with s = 4/((1-eps) lam_max^2), c1 = -2(1+eps)/(1-eps).  A sign apply
// costs 2n+1 applications of D_w and five spinor vectors.
//
// The projection reads the FP64 eigenvectors twice: pass 1 forms
// C = V^dag Psi (FP64 accumulation, deterministic two-stage reduction);
// pass 2 forms psi_h = psi - V C and w = V (sign(lambda) C) in one sweep.
#include <algorithm>
#include <cmath>

#include "ops.h"

struct ovl_sign {
  double lam_max;
  double eps;
  double delta;  // measured max |1 - sqrt(x) P(x)| on [eps, 1]
  std::vector<double> c;  // c_0..c_n, c_0 already halved
};

struct ovl_lowmodes {
  ovl_geom geom;
  int ell;
  const void* V;              // borrowed: ell FP64 spinors
  std::vector<double> lambda;
  double* dev_sign = nullptr;  // sign(lambda_i) on the device
};

namespace ovl {

// ------------------------------------------------------------ coefficients
// Chebyshev interpolation of x^{-1/2} on [eps, 1] at the n+1 Chebyshev-Gauss
// nodes of y; c_k = 2/(n+1) sum_j f(x_j) cos(k theta_j), c_0 halved.
std::vector<double> cheb_coeffs(double eps, int n) {
  std::vector<double> f(n + 1), c(n + 1);
  const double pi = 3.14159265358979323846;
  for (int j = 0; j <= n; ++j) {
    const double th = pi * (j + 0.5) / (n + 1);
    const double x = 0.5 * ((1.0 - eps) * std::cos(th) + 1.0 + eps);
    f[j] = 1.0 / std::sqrt(x);
  }
  for (int k = 0; k <= n; ++k) {
    double s = 0.0;
    for (int j = 0; j <= n; ++j) s += f[j] * std::cos(k * pi * (j + 0.5) / (n + 1));
    c[k] = 2.0 / (n + 1) * s;
  }
  c[0] *= 0.5;
  return c;
}

// max |1 - sqrt(x) P(x)| over npts points of [eps, 1]: half uniform in x,
// half at cos(theta) for theta uniform in [0, pi] (dense near both ends).
double sign_delta(const std::vector<double>& c, double eps, int npts = 400000) {
  const int half = npts / 2, rest = npts - half;
  const double pi = 3.14159265358979323846;
  double worst = 0.0;
  auto eval = [&](double x) {
    const double y = (2.0 * x - 1.0 - eps) / (1.0 - eps);
    double b1 = 0.0, b2 = 0.0;  // Clenshaw in y
    for (int k = static_cast<int>(c.size()) - 1; k >= 1; --k) {
      const double b = c[k] + 2.0 * y * b1 - b2;
      b2 = b1;
      b1 = b;
    }
    const double p = c[0] + y * b1 - b2;
    const double d = std::fabs(1.0 - std::sqrt(x) * p);
    if (d > worst || d != d) worst = (d != d) ? INFINITY : d;
  };
  for (int i = 0; i < half; ++i) eval(half == 1 ? eps : eps + (1.0 - eps) * i / (half - 1));
  for (int i = 0; i < rest; ++i) {
    const double th = rest == 1 ? 0.0 : pi * i / (rest - 1);
    eval(0.5 * ((1.0 - eps) * std::cos(th) + 1.0 + eps));
  }
  return worst;
}

// Smallest n with measured delta <= target, searched from the order law
// delta = 0.41 exp(-2.1 n sqrt(eps)) (eq. 11): bracket, then bisect.
int sign_order(double eps, double target) {
  auto ok = [&](int n) { return sign_delta(cheb_coeffs(eps, n), eps) <= target; };
  int n0 = static_cast<int>(std::ceil(std::log(0.41 / target) / (2.1 * std::sqrt(eps))));
  n0 = std::max(n0, 1);
  int lo, hi;
  if (ok(n0)) {
    hi = n0;
    int step = 1;
    lo = n0 - step;
    while (lo >= 1 && ok(lo)) {
      hi = lo;
      step *= 2;
      lo = hi - step;
    }
    lo = std::max(lo, 0);
  } else {
    lo = n0;
    int step = 1;
    hi = n0 + step;
    while (!ok(hi)) {
      lo = hi;
      step *= 2;
      hi = lo + step;
      OVL_REQUIRE(hi <= 20000, OVL_E_ARG, "sign approximation needs order > 20000");
    }
  }
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (ok(mid)) hi = mid;
    else lo = mid;
  }
  return hi;
}

namespace {

// ------------------------------------------------------------- projection
// Elements are walked in "rows" (parity p, complex index c): 24 rows of Nh
// sites, so each complex of a vector is addressed the same way in every
// storage precision.
template <int P>
__device__ inline size_t cx_offset(int row, int h, int Nh) {
  constexpr int cpb = Prec<P>::cpb;
  const int p = row / 12, c = row % 12;
  const size_t blk = (static_cast<size_t>(p) * (12 / cpb) + c / cpb) * Nh + h;
  return blk * 16 + (c % cpb) * (16 / cpb);
}

template <int P>
__device__ inline Cx<double> load_cx(const char* base, int row, int h, int Nh) {
  Cx<typename Prec<P>::real> v = ScalarIO<P>::load1(base + cx_offset<P>(row, h, Nh));
  return {static_cast<double>(v.re), static_cast<double>(v.im)};
}

template <int P>
__device__ inline void store_cx(char* base, int row, int h, int Nh, Cx<double> v) {
  using real = typename Prec<P>::real;
  ScalarIO<P>::store1(base + cx_offset<P>(row, h, Nh), Cx<real>{static_cast<real>(v.re), static_cast<real>(v.im)});
}

constexpr int PJ_TILE = 64;     // elements per tile (one per lane)
constexpr int PJ_WAVES = 8;     // waves per block in pass 1
constexpr int PJ_BLOCKS = 512;  // K-split of pass 1

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Pass 1: partial[(i*G + b)*R + r] = sum over block b's tiles of conj(V_i) Psi_r.
// blockIdx.y selects a group of PJ_WAVES*IW eigenvectors; each wave owns IW.
template <int PP, int RMAX, int IW>
__global__ __launch_bounds__(PJ_WAVES * 64) void proj_dot_kernel(int Nh, int ell, const char* V, size_t vstrideV,
                                                                  const char* psi, size_t vstrideP, int R,
                                                                  double2* partial) {
  __shared__ Cx<double> tile[RMAX][PJ_TILE];
  const int tiles_per_row = (Nh + PJ_TILE - 1) / PJ_TILE;
  const long total = 24L * tiles_per_row;
  const long t0 = total * blockIdx.x / gridDim.x, t1 = total * (blockIdx.x + 1) / gridDim.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ibase = (blockIdx.y * PJ_WAVES + wave) * IW;
  Cx<double> acc[IW][RMAX];
#pragma unroll
  for (int j = 0; j < IW; ++j)
#pragma unroll
    for (int r = 0; r < RMAX; ++r) acc[j][r] = {0.0, 0.0};

  for (long t = t0; t < t1; ++t) {
    const int row = static_cast<int>(t / tiles_per_row);
    const int h0 = static_cast<int>(t % tiles_per_row) * PJ_TILE;
    __syncthreads();
    for (int k = threadIdx.x; k < R * PJ_TILE; k += blockDim.x) {
      const int r = k / PJ_TILE, l = k % PJ_TILE;
      tile[r][l] = (h0 + l < Nh) ? load_cx<PP>(psi + r * vstrideP, row, h0 + l, Nh) : Cx<double>{0.0, 0.0};
    }
    __syncthreads();
    const int h = h0 + lane;
    if (h < Nh) {
      Cx<double> ps[RMAX];
#pragma unroll
      for (int r = 0; r < RMAX; ++r) ps[r] = (r < R) ? tile[r][lane] : Cx<double>{0.0, 0.0};
#pragma unroll
      for (int j = 0; j < IW; ++j) {
        const int i = ibase + j;
        if (i < ell) {
          const Cx<double> v = load_cx<OVL_F64>(V + i * vstrideV, row, h, Nh);
#pragma unroll
          for (int r = 0; r < RMAX; ++r) acc[j][r] = acc[j][r] + cmul_conj(v, ps[r]);
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < IW; ++j) {
    const int i = ibase + j;
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      const double re = wsum(acc[j][r].re), im = wsum(acc[j][r].im);
      if (lane == 0 && i < ell && r < R)
        partial[(static_cast<size_t>(i) * gridDim.x + blockIdx.x) * R + r] = make_double2(re, im);
    }
  }
}

// C[i*R + r] = sum_b partial[(i*G + b)*R + r], in block order.
__global__ void proj_reduce_kernel(int ell, int R, int G, const double2* partial, double2* C) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ell * R) return;
  const int i = k / R, r = k % R;
  double re = 0.0, im = 0.0;
  for (int b = 0; b < G; ++b) {
    const double2 v = partial[(static_cast<size_t>(i) * G + b) * R + r];
    re += v.x;
    im += v.y;
  }
  C[k] = make_double2(re, im);
}

// Pass 2: psi_h = psi - sum_i C_i eta_i, w = G5? sum_i sign_i C_i eta_i.
// One thread per element; coefficients staged in LDS (broadcast reads).
template <int PP, int RMAX>
__global__ __launch_bounds__(256) void proj_update_kernel(int Nh, int ell, const char* V, size_t vstrideV,
                                                          const char* psi, char* psih, char* w, size_t vstrideP,
                                                          int R, const double2* C, const double* sgn, int g5w) {
  extern __shared__ double2 coef[];  // [ell][R] of C, then [ell] signs folded in at use
  for (int k = threadIdx.x; k < ell * R; k += blockDim.x) coef[k] = C[k];
  __syncthreads();
  const int row = blockIdx.y;
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= Nh) return;
  Cx<double> ph[RMAX], ww[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    ph[r] = (r < R) ? load_cx<PP>(psi + r * vstrideP, row, h, Nh) : Cx<double>{0.0, 0.0};
    ww[r] = {0.0, 0.0};
  }
  for (int i = 0; i < ell; ++i) {
    const Cx<double> v = load_cx<OVL_F64>(V + i * vstrideV, row, h, Nh);
    const double s = sgn[i];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      if (r < R) {
        const double2 cc = coef[i * R + r];
        const Cx<double> vc = v * Cx<double>{cc.x, cc.y};
        ph[r] = ph[r] - vc;
        ww[r] = ww[r] + s * vc;
      }
    }
  }
  const double gs = (g5w && (row % 12) >= 6) ? -1.0 : 1.0;  // spin 2,3 of gamma5
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    if (r < R) {
      store_cx<PP>(psih + r * vstrideP, row, h, Nh, ph[r]);
      store_cx<PP>(w + r * vstrideP, row, h, Nh, gs * ww[r]);
    }
  }
}

template <int PP, int RMAX, int IW>
void proj_launch(const ovl_lowmodes* lm, const void* psi, void* psih, void* w, int R, int g5w, hipStream_t s) {
  const ovl_geom* g = &lm->geom;
  const int Nh = g->geo.Nh, ell = lm->ell;
  const size_t vsV = spinor_vec_bytes(g, OVL_F64), vsP = spinor_vec_bytes(g, PP);
  const int groups = (ell + PJ_WAVES * IW - 1) / (PJ_WAVES * IW);
  WsBuf part(static_cast<size_t>(ell) * PJ_BLOCKS * R * sizeof(double2), s);
  WsBuf cbuf(static_cast<size_t>(ell) * R * sizeof(double2), s);
  hipLaunchKernelGGL((proj_dot_kernel<PP, RMAX, IW>), dim3(PJ_BLOCKS, groups), dim3(PJ_WAVES * 64), 0, s, Nh, ell,
                     static_cast<const char*>(lm->V), vsV, static_cast<const char*>(psi), vsP, R,
                     static_cast<double2*>(part.p));
  OVL_HIP(hipGetLastError());
  hipLaunchKernelGGL(proj_reduce_kernel, dim3((ell * R + 255) / 256), dim3(256), 0, s, ell, R, PJ_BLOCKS,
                     static_cast<const double2*>(part.p), static_cast<double2*>(cbuf.p));
  OVL_HIP(hipGetLastError());
  const size_t lds = static_cast<size_t>(ell) * R * sizeof(double2);
  OVL_REQUIRE(lds <= 64 * 1024, OVL_E_ARG, "projection: ell * nrhs too large (max 4096)");
  hipLaunchKernelGGL((proj_update_kernel<PP, RMAX>), dim3((Nh + 255) / 256, 24), dim3(256), lds, s, Nh, ell,
                     static_cast<const char*>(lm->V), vsV, static_cast<const char*>(psi), static_cast<char*>(psih),
                     static_cast<char*>(w), vsP, R, static_cast<const double2*>(cbuf.p), lm->dev_sign, g5w);
  OVL_HIP(hipGetLastError());
}

template <int PP>
void proj_rmax(const ovl_lowmodes* lm, const void* psi, void* psih, void* w, int R, int g5w, hipStream_t s) {
  if (R == 1) proj_launch<PP, 1, 8>(lm, psi, psih, w, R, g5w, s);
  else if (R <= 4) proj_launch<PP, 4, 4>(lm, psi, psih, w, R, g5w, s);
  else proj_launch<PP, 12, 2>(lm, psi, psih, w, R, g5w, s);
}

}  // namespace

// psi_h and w for a batch of nrhs spinors (precision prec); w gets gamma5
// applied when g5w is set.  psi may not alias psi_h or w.
void lowmode_project(const ovl_lowmodes* lm, const void* psi, void* psih, void* w, int prec, int nrhs, int g5w,
                     hipStream_t s) {
  OVL_REQUIRE(nrhs <= OVL_MAX_RHS, OVL_E_ARG, "projection supports at most 12 right-hand sides");
  switch (prec) {
    case OVL_F64: proj_rmax<OVL_F64>(lm, psi, psih, w, nrhs, g5w, s); break;
    case OVL_F32: proj_rmax<OVL_F32>(lm, psi, psih, w, nrhs, g5w, s); break;
    case OVL_F16: proj_rmax<OVL_F16>(lm, psi, psih, w, nrhs, g5w, s); break;
    case OVL_BF16: proj_rmax<OVL_BF16>(lm, psi, psih, w, nrhs, g5w, s); break;
  }
}

// ------------------------------------------------------------- Clenshaw
namespace {

// A Clenshaw iterate b = v + a * psi_h (v may be null).
struct Term {
  void* v;
  double a;
};

struct Stencil {
  const ovl_gauge* u;
  const void* links;
  int recon, prec, nrhs;
  double rho;
  hipStream_t s;
  size_t vstride;

  // out = scale * G(D_w(-rho) in) + sum_j cv_j G_j(v_j)
  void apply(void* out, const void* in, double scale, int g5, std::initializer_list<const void*> vs,
             std::initializer_list<double> cs, int g5v = 0) const {
    StencilArgs A{};
    A.g = u->geom.geo;
    A.out = out;
    A.in = in;
    A.links = links;
    A.a = scale * (4.0 - rho);
    A.b = -0.5 * scale;
    A.g5 = g5;
    A.g5v = g5v;
    A.par0 = 0;
    A.npar = 2;
    A.vstride = vstride;
    int j = 0;
    auto ci = cs.begin();
    for (const void* v : vs) {
      A.v[j] = v;
      A.cv[j] = *ci++;
      ++j;
    }
    A.nv = j;
    launch_stencil(A, prec, recon, nrhs, s);
  }
};

}  // namespace

// out = Q P(Q^2) psi_h  + lowpart-combine, i.e. the last launch is
//   out = fscale * G_f(D_w(-rho) P) + sum_j fc_j G_j(fv_j)
// (see the callers for the combinations used).  Workspace: 3 vectors.
void clenshaw_sign(const Stencil& st, const ovl_sign* sg, const void* psih, void* out, double fscale, int fg5,
                   const void* fv0, double fc0, const void* fv1, double fc1, int fg5v) {
  const double eps = sg->eps, lam = sg->lam_max;
  const double s2 = 4.0 / ((1.0 - eps) * lam * lam);  // 2Y = s2 H_w H_w + c1
  const double c1 = -2.0 * (1.0 + eps) / (1.0 - eps);
  const int n = static_cast<int>(sg->c.size()) - 1;
  const std::vector<double>& c = sg->c;
  const size_t vb = st.vstride * st.nrhs;
  WsBuf bufA(vb, st.s), bufB(vb, st.s), tbuf(vb, st.s);
  void* t = tbuf.p;
  Term b1{nullptr, 0.0}, b2{nullptr, 0.0};  // b_{k+1}, b_{k+2}
  void* freebuf[2] = {bufA.p, bufB.p};

  // one Clenshaw step with weight f on the 2Y part:
  //   out = f*2Y(b1) - b2 + cpsi*psi_h  written to dst
  auto step = [&](void* dst, double f, double cpsi) {
    if (b1.v == nullptr) {
      // b1 = a psi_h:  f*2Y(a psi_h) = f*a*s2 H H psi_h + f*a*c1 psi_h
      st.apply(t, psih, 1.0, 1, {}, {});
      const double cp = cpsi + f * b1.a * c1 - b2.a;
      if (b2.v)
        st.apply(dst, t, f * b1.a * s2, 1, {psih, b2.v}, {cp, -1.0});
      else
        st.apply(dst, t, f * b1.a * s2, 1, {psih}, {cp});
    } else {
      st.apply(t, b1.v, 1.0, 1, {}, {});
      const double cp = cpsi - b2.a;
      if (b2.v)
        st.apply(dst, t, f * s2, 1, {b1.v, b2.v, psih}, {f * c1, -1.0, cp});
      else
        st.apply(dst, t, f * s2, 1, {b1.v, psih}, {f * c1, cp});
    }
  };

  for (int k = n; k >= 1; --k) {
    if (b1.v == nullptr && b1.a == 0.0) {  // k == n: b_n = c_n psi_h, kept implicit
      b2 = b1;
      b1 = Term{nullptr, c[k]};
      continue;
    }
    // write over b_{k+2}'s buffer when it has one (same-site read before write)
    void* dst = b2.v ? b2.v : (b1.v == freebuf[0] ? freebuf[1] : freebuf[0]);
    step(dst, 1.0, c[k]);
    b2 = b1;
    b1 = Term{dst, 0.0};
  }
  // P psi_h = c_0 psi_h + Y b_1 - b_2
  void* pbuf;
  if (n == 0) {
    // P = c_0: the final launch applies to c_0 psi_h
    pbuf = nullptr;
  } else {
    pbuf = b2.v ? b2.v : (b1.v == freebuf[0] ? freebuf[1] : freebuf[0]);
    step(pbuf, 0.5, c[0]);
  }
  // final: out = fscale * G_f(D_w(-rho) P) + extras
  const void* pin = pbuf ? pbuf : psih;
  const double sc = pbuf ? fscale : fscale * c[0];
  if (fv0 && fv1)
    st.apply(out, pin, sc, fg5, {fv0, fv1}, {fc0, fc1}, fg5v);
  else if (fv0)
    st.apply(out, pin, sc, fg5, {fv0}, {fc0}, fg5v);
  else
    st.apply(out, pin, sc, fg5, {}, {});
}

// Overlap-operator driver.  mode: 0 = sign(H_w) in, 1 = D(m) in, 2 = D(m)^dag in.
void overlap_apply(void* out, const void* in, const ovl_gauge* u, double rho, double m, const ovl_sign* sg,
                   const ovl_lowmodes* lm, int mode, int prec, int nrhs, hipStream_t s) {
  Stencil st;
  st.u = u;
  st.links = gauge_links(u, prec, &st.recon);
  st.prec = prec;
  st.nrhs = nrhs;
  st.rho = rho;
  st.s = s;
  st.vstride = spinor_vec_bytes(&u->geom, prec);
  const size_t vb = st.vstride * nrhs;
  const double lam = sg->lam_max;

  // the sign function acts on src = in (mode 0, 1) or gamma5 in (mode 2)
  const void* src = in;
  WsBuf g5buf(mode == 2 ? vb : 16, s);
  if (mode == 2) {
    blas_gamma5(prec, st.vstride, in, g5buf.p, nrhs, s);
    src = g5buf.p;
  }
  const void* psih = src;
  WsBuf hbuf(lm ? vb : 16, s), wbuf(lm ? vb : 16, s);
  const void* w = nullptr;
  // mode 1 needs gamma5 w in the combine; fold it into the projection
  if (lm) {
    lowmode_project(lm, src, hbuf.p, wbuf.p, prec, nrhs, mode == 1 ? 1 : 0, s);
    psih = hbuf.p;
    w = wbuf.p;
  }
  const double ap = rho + 0.5 * m, am = rho - 0.5 * m;
  if (mode == 0) {
    // sign = (1/lam) H_w P + w
    clenshaw_sign(st, sg, psih, out, 1.0 / lam, 1, w, 1.0, nullptr, 0.0, 0);
  } else if (mode == 1) {
    // D(m) in = ap in + am gamma5 (H_w P / lam + w) = (am/lam) D_w P + ap in + am gamma5 w
    clenshaw_sign(st, sg, psih, out, am / lam, 0, in, ap, w, am, 0);
  } else {
    // D(m)^dag in = ap in + am sign(gamma5 in) = (am/lam) H_w P + ap in + am w
    clenshaw_sign(st, sg, psih, out, am / lam, 1, in, ap, w, am, 0);
  }
}

}  // namespace ovl

using namespace ovl;

extern "C" {

int ovl_sign_create(double lam_lo, double lam_max, double delta, int n, ovl_sign** out) {
  return guard([&] {
    OVL_REQUIRE(out, OVL_E_ARG, "null argument");
    OVL_REQUIRE(lam_lo > 0.0 && lam_max > lam_lo && std::isfinite(lam_max), OVL_E_ARG,
                "need 0 < lam_lo < lam_max");
    OVL_REQUIRE(n >= 0 && n <= 20000, OVL_E_ARG, "order out of range");
    OVL_REQUIRE(n > 0 || (delta > 0.0 && delta < 1.0), OVL_E_ARG, "need 0 < delta < 1 when n = 0");
    const double eps = (lam_lo / lam_max) * (lam_lo / lam_max);
    const int order = n > 0 ? n : sign_order(eps, delta);
    ovl_sign* sg = new ovl_sign;
    sg->lam_max = lam_max;
    sg->eps = eps;
    sg->c = cheb_coeffs(eps, order);
    sg->delta = sign_delta(sg->c, eps);
    *out = sg;
    return OVL_OK;
  });
}

int ovl_sign_destroy(ovl_sign* s) {
  delete s;
  return OVL_OK;
}

int ovl_sign_info(const ovl_sign* s, int* n, double* eps, double* delta) {
  return guard([&] {
    OVL_REQUIRE(s, OVL_E_ARG, "null argument");
    if (n) *n = static_cast<int>(s->c.size()) - 1;
    if (eps) *eps = s->eps;
    if (delta) *delta = s->delta;
    return OVL_OK;
  });
}

int ovl_sign_coeffs(const ovl_sign* s, double* c, int cap) {
  return guard([&] {
    OVL_REQUIRE(s && c, OVL_E_ARG, "null argument");
    OVL_REQUIRE(cap >= static_cast<int>(s->c.size()), OVL_E_ARG, "coefficient buffer too small");
    std::copy(s->c.begin(), s->c.end(), c);
    return OVL_OK;
  });
}

int ovl_lowmodes_create(const ovl_geom* g, int ell, const void* V, const double* lambda, ovl_lowmodes** out) {
  return guard([&] {
    OVL_REQUIRE(g && out && (ell == 0 || (V && lambda)), OVL_E_ARG, "null argument");
    OVL_REQUIRE(ell >= 0 && ell <= 4096, OVL_E_ARG, "ell out of range");
    ovl_lowmodes* lm = new ovl_lowmodes;
    lm->geom = *g;
    lm->ell = ell;
    lm->V = V;
    lm->lambda.assign(lambda, lambda + ell);
    std::vector<double> sg(std::max(ell, 1));
    for (int i = 0; i < ell; ++i) {
      if (!std::isfinite(lambda[i])) {
        delete lm;
        throw Error(OVL_E_NAN, "non-finite eigenvalue");
      }
      sg[i] = lambda[i] >= 0.0 ? 1.0 : -1.0;
    }
    if (hipMalloc(&lm->dev_sign, sg.size() * sizeof(double)) != hipSuccess) {
      delete lm;
      throw Error(OVL_E_NOMEM, "lowmodes: device allocation failed");
    }
    OVL_HIP(hipMemcpy(lm->dev_sign, sg.data(), sg.size() * sizeof(double), hipMemcpyHostToDevice));
    *out = lm;
    return OVL_OK;
  });
}

int ovl_lowmodes_destroy(ovl_lowmodes* lm) {
  if (lm) {
    if (lm->dev_sign) (void)hipFree(lm->dev_sign);
    delete lm;
  }
  return OVL_OK;
}

int ovl_lowmodes_project(const ovl_lowmodes* lm, const void* in, void* psi_h, void* w, ovl_prec prec, int nrhs,
                         ovl_stream_t s) {
  return guard([&] {
    OVL_REQUIRE(lm && in && psi_h && w, OVL_E_ARG, "null argument");
    check_prec(prec);
    check_nrhs(nrhs);
    OVL_REQUIRE(lm->ell > 0, OVL_E_ARG, "no low modes");
    OVL_REQUIRE(in != psi_h && in != w && psi_h != w, OVL_E_ALIAS, "projection outputs must not alias");
    lowmode_project(lm, in, psi_h, w, prec, nrhs, 0, static_cast<hipStream_t>(s));
    return OVL_OK;
  });
}

static void overlap_common(void* out, const void* in, const ovl_gauge* u, const ovl_sign* sg,
                           const ovl_lowmodes* lm, int prec, int nrhs) {
  OVL_REQUIRE(out && in && u && sg, OVL_E_ARG, "null argument");
  check_prec(prec);
  check_nrhs(nrhs);
  OVL_REQUIRE(out != in, OVL_E_ALIAS, "output must not alias the input");
  if (lm) {
    OVL_REQUIRE(lm->geom.N == u->geom.N, OVL_E_ARG, "low modes and gauge field have different lattices");
    OVL_REQUIRE(out != lm->V, OVL_E_ALIAS, "output aliases the eigenvectors");
    if (lm->ell == 0) lm = nullptr;
  }
}

int ovl_sign_apply(void* out, const void* in, const ovl_gauge* u, double rho, const ovl_sign* sg,
                   const ovl_lowmodes* lm, ovl_prec prec, int nrhs, ovl_stream_t s) {
  return guard([&] {
    overlap_common(out, in, u, sg, lm, prec, nrhs);
    overlap_apply(out, in, u, rho, 0.0, sg, (lm && lm->ell) ? lm : nullptr, 0, prec, nrhs,
                  static_cast<hipStream_t>(s));
    return OVL_OK;
  });
}

int ovl_overlap_apply(void* out, const void* in, const ovl_gauge* u, double rho, double m, const ovl_sign* sg,
                      const ovl_lowmodes* lm, int dagger, ovl_prec prec, int nrhs, ovl_stream_t s) {
  return guard([&] {
    overlap_common(out, in, u, sg, lm, prec, nrhs);
    OVL_REQUIRE(dagger == 0 || dagger == 1, OVL_E_ARG, "dagger must be 0 or 1");
    overlap_apply(out, in, u, rho, m, sg, (lm && lm->ell) ? lm : nullptr, dagger ? 2 : 1, prec, nrhs,
                  static_cast<hipStream_t>(s));
    return OVL_OK;
  });
}

}  // extern "C"
