// Rational sign function (arXiv:1106.4964 Sec. II eq. 4-5, Sec. V eq. 12):
// the comparison variants of the polynomial sign.
//
//   sign(H_w) psi = sum_i sign(lambda_i) (eta_i^dag psi) eta_i + Q P(Q^2) psi_h,
//   P(y) = sum_l b_l / (y + c_l),  y = Q^2 = (H_w / lam_max)^2,
//
// with P the optimal (Zolotarev) rational approximation of y^{-1/2} of type
// (n-1, n) on [eps, 1].  P(Q^2) psi_h is evaluated two ways:
//  * single pass: a multi-shift CG solves (Q^2 + c_l) x_l = psi_h for all l
//    in one Krylov space (2n + 3 FP64 vectors); the shifted directions and
//    iterates are updated by one fused kernel that reads the base residual
//    once for every shift;
//  * double pass: a Lanczos pass on Q^2 builds the tridiagonal T_k until the
//    coefficients y = P(T_k) e_1 have converged, and a second pass rebuilds
//    the same Lanczos vectors and sums y_j v_j (six vectors, independent of
//    n, twice the applications of Q^2).
// Each application of Q^2 is two stencil launches, the second one adding
// the base shift through the fused epilogue.  Everything is FP64; the
// Krylov scalars go through the host once or twice per iteration.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>

#include "ops.h"

namespace ovl {
namespace {

constexpr double kPi = 3.14159265358979323846;

// Complete elliptic integral of the first kind, parameter m = k^2, by the
// arithmetic-geometric mean: K = pi / (2 AGM(1, sqrt(1 - m))).
double ellip_k(double m) {
  double a = 1.0, b = std::sqrt(1.0 - m);
  for (int i = 0; i < 64 && std::fabs(a - b) > 1e-16 * a; ++i) {
    const double an = 0.5 * (a + b);
    b = std::sqrt(a * b);
    a = an;
  }
  return kPi / (2.0 * a);
}

// Jacobi amplitude phi(u | m) by the descending AGM (Abramowitz & Stegun
// 16.4): sn = sin(phi), cn = cos(phi).
double jacobi_am(double u, double m) {
  double a[64], c[64];
  a[0] = 1.0;
  c[0] = std::sqrt(m);
  double b = std::sqrt(1.0 - m);
  int N = 0;
  while (N < 63 && std::fabs(c[N]) > 1e-16) {
    a[N + 1] = 0.5 * (a[N] + b);
    c[N + 1] = 0.5 * (a[N] - b);
    b = std::sqrt(a[N] * b);
    ++N;
  }
  double phi = std::ldexp(a[N] * u, N);
  for (int k = N; k > 0; --k) phi = 0.5 * (phi + std::asin(c[k] * std::sin(phi) / a[k]));
  return phi;
}

}  // namespace
}  // namespace ovl

// Optimal rational approximation of y^{-1/2} on [eps, 1] (partial fractions).
struct ovl_rational {
  double lam_max;
  double eps;
  double delta;           // measured max |1 - sqrt(y) P(y)|
  std::vector<double> b;  // residues
  std::vector<double> c;  // shifts (poles at -c)
};

namespace ovl {
namespace {

// Zolotarev's closed form on x in [1, B], B = 1/eps: d0 prod_{l<n}(x + s_{2l})
// / prod_{l<=n}(x + s_{2l-1}), s_j = sn^2/cn^2 (j K'/(2n) | 1 - 1/B); d0 from
// the equal-ripple condition on a log-uniform grid; then partial fractions in
// y = x / B.
void zolotarev(double eps, int n, ovl_rational* r) {
  const double B = 1.0 / eps, mp = 1.0 - eps;
  const double Kp = ellip_k(mp);
  std::vector<double> s(2 * n);  // s[1..2n-1]
  for (int j = 1; j < 2 * n; ++j) {
    const double t = std::tan(jacobi_am(j * Kp / (2 * n), mp));
    s[j] = t * t;
  }
  std::vector<double> num, den;
  for (int j = 1; j < 2 * n; ++j) (j % 2 ? den : num).push_back(s[j]);
  const int npts = 200001;
  const double l0 = 0.0, l1 = std::log(B);
  auto prod = [&](double x) {
    double p = 1.0;
    for (double v : num) p *= x + v;
    for (double v : den) p /= x + v;
    return p;
  };
  double fmax = -INFINITY, fmin = INFINITY;
  for (int i = 0; i < npts; ++i) {
    const double x = std::exp(l0 + (l1 - l0) * i / (npts - 1));
    const double f = std::sqrt(x) * prod(x);
    fmax = std::max(fmax, f);
    fmin = std::min(fmin, f);
  }
  const double d0 = 2.0 / (fmax + fmin);
  r->b.assign(n, 0.0);
  r->c.assign(n, 0.0);
  for (int l = 0; l < n; ++l) {
    const double p = -den[l];
    double a = 1.0;
    for (double v : num) a *= v + p;
    for (int i = 0; i < n; ++i)
      if (i != l) a /= den[i] + p;
    r->b[l] = d0 * a / std::sqrt(B);
    r->c[l] = den[l] / B;
  }
  double worst = 0.0;
  for (int i = 0; i < npts; ++i) {
    const double y = std::exp(std::log(eps) * (1.0 - static_cast<double>(i) / (npts - 1)));
    double pv = 0.0;
    for (int l = 0; l < n; ++l) pv += r->b[l] / (y + r->c[l]);
    worst = std::max(worst, std::fabs(1.0 - std::sqrt(y) * pv));
  }
  r->delta = worst;
}

// For each 16-byte FP64 element and every active shift l:
//   x_l += alpha_l p_l,   p_l = zeta_l r + beta_l p_l
// coef[4 l + (0, 1, 2, 3)] = (alpha_l, zeta_l, beta_l, active_l).
__global__ void shift_update_kernel(size_t n16, int n, const double2* __restrict__ r, double2* X, double2* Pm,
                                    size_t vs16, const double* __restrict__ coef) {
  const size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (e >= n16) return;
  const double2 rv = r[e];
  for (int l = 0; l < n; ++l) {
    if (coef[4 * l + 3] == 0.0) continue;
    const double al = coef[4 * l], ze = coef[4 * l + 1], be = coef[4 * l + 2];
    const size_t o = l * vs16 + e;
    const double2 pv = Pm[o];
    double2 xv = X[o];
    xv.x = fma(al, pv.x, xv.x);
    xv.y = fma(al, pv.y, xv.y);
    X[o] = xv;
    Pm[o] = make_double2(fma(ze, rv.x, be * pv.x), fma(ze, rv.y, be * pv.y));
  }
}

// One rebuilt Lanczos step of the second pass, in place over three vectors:
//   w = (Q^2 v) - beta_prev v_prev - alpha v  (w holds Q^2 v on entry),
//   v_prev <- v,  v <- w / beta,  out += y v
__global__ void lanczos_step_kernel(size_t n16, double2* w, double2* v, double2* vp, double2* out, double alpha,
                                    double beta_prev, double inv_beta, double y) {
  const size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (e >= n16) return;
  const double2 a = w[e], vv = v[e], pp = vp[e];
  const double2 nv = make_double2((a.x - beta_prev * pp.x - alpha * vv.x) * inv_beta,
                                  (a.y - beta_prev * pp.y - alpha * vv.y) * inv_beta);
  vp[e] = vv;
  v[e] = nv;
  double2 o = out[e];
  o.x = fma(y, nv.x, o.x);
  o.y = fma(y, nv.y, o.y);
  out[e] = o;
}

// y = sum_l b_l (T + c_l)^{-1} e_1 for the k x k symmetric tridiagonal T
// (diagonal al, off-diagonal be[0..k-2]) by Thomas elimination per shift
// (T + c_l is positive definite).
std::vector<double> tridiag_rational_e1(const std::vector<double>& al, const std::vector<double>& be,
                                        const ovl_rational* r) {
  const int k = static_cast<int>(al.size());
  std::vector<double> y(k, 0.0), d(k), z(k);
  for (size_t l = 0; l < r->c.size(); ++l) {
    // forward elimination of (T + c) z = e_1
    d[0] = al[0] + r->c[l];
    z[0] = 1.0;
    for (int i = 1; i < k; ++i) {
      const double f = be[i - 1] / d[i - 1];
      d[i] = al[i] + r->c[l] - f * be[i - 1];
      z[i] = -f * z[i - 1];
    }
    z[k - 1] /= d[k - 1];
    for (int i = k - 2; i >= 0; --i) z[i] = (z[i] - be[i] * z[i + 1]) / d[i];
    for (int i = 0; i < k; ++i) y[i] += r->b[l] * z[i];
  }
  return y;
}

struct DevVec {
  void* p = nullptr;
  size_t n = 0;
  explicit DevVec(size_t bytes) : n(bytes) {
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(OVL_E_NOMEM, "rational sign: device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    mem_track(static_cast<int64_t>(n));
  }
  ~DevVec() {
    if (p) {
      (void)hipFree(p);
      mem_track(-static_cast<int64_t>(n));
    }
  }
  DevVec(const DevVec&) = delete;
  DevVec& operator=(const DevVec&) = delete;
};

}  // namespace
}  // namespace ovl

using namespace ovl;

extern "C" {

int ovl_rational_create(double lam_lo, double lam_max, int n, ovl_rational** out) {
  return guard([&] {
    OVL_REQUIRE(out, OVL_E_ARG, "null argument");
    OVL_REQUIRE(lam_lo > 0.0 && lam_max > lam_lo && std::isfinite(lam_max), OVL_E_ARG, "need 0 < lam_lo < lam_max");
    OVL_REQUIRE(n >= 1 && n <= 32, OVL_E_ARG, "need 1 <= n <= 32 partial fractions");
    ovl_rational* r = new ovl_rational;
    r->lam_max = lam_max;
    r->eps = (lam_lo / lam_max) * (lam_lo / lam_max);
    zolotarev(r->eps, n, r);
    *out = r;
    return OVL_OK;
  });
}

int ovl_rational_destroy(ovl_rational* r) {
  delete r;
  return OVL_OK;
}

int ovl_rational_coeffs(const ovl_rational* r, double* b, double* c, int cap, double* eps, double* delta) {
  return guard([&] {
    OVL_REQUIRE(r && b && c, OVL_E_ARG, "null argument");
    OVL_REQUIRE(cap >= static_cast<int>(r->c.size()), OVL_E_ARG, "coefficient buffer too small");
    std::copy(r->b.begin(), r->b.end(), b);
    std::copy(r->c.begin(), r->c.end(), c);
    if (eps) *eps = r->eps;
    if (delta) *delta = r->delta;
    return static_cast<int>(r->c.size());
  });
}

int ovl_rational_sign_apply(void* out, const void* in, const ovl_gauge* u, double rho, const ovl_rational* rat,
                            const ovl_lowmodes* lm, int method, double tol, int maxiter, ovl_rational_stats* stats,
                            ovl_stream_t st) {
  return guard([&] {
    OVL_REQUIRE(out && in && u && rat && stats, OVL_E_ARG, "null argument");
    OVL_REQUIRE(out != in, OVL_E_ALIAS, "output must not alias the input");
    OVL_REQUIRE(method == 0 || method == 1, OVL_E_ARG, "method: 0 multi-shift CG, 1 double pass");
    OVL_REQUIRE(tol > 0.0 && maxiter >= 1, OVL_E_ARG, "need tol > 0 and maxiter >= 1");
    if (lm && lm->ell == 0) lm = nullptr;
    if (lm) OVL_REQUIRE(lm->geom.N == u->geom.N, OVL_E_ARG, "low modes and gauge field have different lattices");
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = static_cast<hipStream_t>(st);
    *stats = ovl_rational_stats{};
    const ovl_geom* g = &u->geom;
    const size_t v64 = spinor_vec_bytes(g, OVL_F64), n16 = v64 / 16, N = static_cast<size_t>(g->N);
    const int n = static_cast<int>(rat->c.size());
    int recon = 0;
    const void* links = gauge_links(u, OVL_F64, &recon);
    const double il = 1.0 / rat->lam_max;
    // out = H_w in / lam_max (+ c0 v0): one stencil launch
    auto qapply = [&](void* o, const void* i, const void* v0, double c0) {
      StencilArgs A{};
      A.g = g->geo;
      A.out = o;
      A.in = i;
      A.links = links;
      A.vstride = v64;
      A.a = (4.0 - rho) * il;
      A.b = -0.5 * il;
      A.g5 = 1;
      A.par0 = 0;
      A.npar = 2;
      if (v0) {
        A.nv = 1;
        A.v[0] = v0;
        A.cv[0] = c0;
      }
      launch_stencil(A, OVL_F64, recon, 1, s);
      stats->hw_applies += 1;
    };
    WsBuf sc(sizeof(double) * 8, s);
    double* dsc = static_cast<double*>(sc.p);
    auto dot_re = [&](const void* x, const void* y) {
      blas_dot(OVL_F64, n16, x, y, 1, v64, dsc, s);
      double h[2];
      OVL_HIP(hipMemcpyAsync(h, dsc, sizeof(h), hipMemcpyDeviceToHost, s));
      OVL_HIP(hipStreamSynchronize(s));
      return h[0];
    };
    auto nrm2 = [&](const void* x) {
      blas_norm2(OVL_F64, n16, x, 1, v64, dsc, s);
      double h[2];
      OVL_HIP(hipMemcpyAsync(h, dsc, sizeof(h), hipMemcpyDeviceToHost, s));
      OVL_HIP(hipStreamSynchronize(s));
      return h[0];
    };
    // y = a x + b y (real host scalars; b = 0: y = a x)
    auto axpby = [&](double a, const void* x, double b, void* y) {
      const double h[4] = {a, 0.0, b, 0.0};
      OVL_HIP(hipMemcpyAsync(dsc + 4, h, sizeof(h), hipMemcpyHostToDevice, s));
      blas_axpby(OVL_F64, x, dsc + 4, OVL_F64, y, b != 0.0 ? dsc + 6 : nullptr, N, 1, s);
      OVL_HIP(hipStreamSynchronize(s));  // the host scalars are reused
    };

    // the low modes exactly (w), the rest (psi_h) through P(Q^2)
    WsBuf psih(v64, s), wlow(v64, s), pq(v64, s), t(v64, s);
    if (lm) {
      lowmode_project(lm, in, psih.p, wlow.p, OVL_F64, 1, 0, s);
    } else {
      OVL_HIP(hipMemcpyAsync(psih.p, in, v64, hipMemcpyDeviceToDevice, s));
    }
    const double bn2 = nrm2(psih.p);
    OVL_REQUIRE(std::isfinite(bn2), OVL_E_NAN, "input contains NaN or Inf");
    int rc = OVL_OK;
    if (bn2 == 0.0) {
      blas_zero(pq.p, v64, s);
    } else if (method == 0) {
      // ------------------------------------------------ multi-shift CG
      int base = 0;
      for (int l = 1; l < n; ++l)
        if (rat->c[l] < rat->c[base]) base = l;
      const double s0 = rat->c[base];
      DevVec X(v64 * n), Pm(v64 * n);
      WsBuf r(v64, s), p(v64, s), q(v64, s), cf(sizeof(double) * 4 * n, s);
      blas_zero(X.p, v64 * n, s);
      for (int l = 0; l < n; ++l)
        OVL_HIP(hipMemcpyAsync(static_cast<char*>(Pm.p) + l * v64, psih.p, v64, hipMemcpyDeviceToDevice, s));
      OVL_HIP(hipMemcpyAsync(r.p, psih.p, v64, hipMemcpyDeviceToDevice, s));
      OVL_HIP(hipMemcpyAsync(p.p, psih.p, v64, hipMemcpyDeviceToDevice, s));
      std::vector<double> zeta(n, 1.0), zeta_prev(n, 1.0), zn(n), coef(4 * n);
      std::vector<char> active(n, 1);
      double rr = bn2, alpha_prev = 1.0, beta_prev = 0.0;
      const double bn = std::sqrt(bn2);
      int its = 0, nact = n;
      while (nact > 0) {
        if (its >= maxiter) {
          rc = OVL_W_NOT_CONVERGED;
          break;
        }
        qapply(t.p, p.p, nullptr, 0.0);
        qapply(q.p, t.p, p.p, s0);  // q = (Q^2 + s0) p
        const double pqd = dot_re(p.p, q.p);
        OVL_REQUIRE(std::isfinite(pqd) && pqd > 0.0, OVL_E_NAN, "multi-shift CG: p^dag A p not positive");
        const double alpha = rr / pqd;
        for (int l = 0; l < n; ++l) {
          if (!active[l]) continue;
          const double sig = rat->c[l] - s0;
          const double den =
              alpha * beta_prev * (zeta_prev[l] - zeta[l]) + zeta_prev[l] * alpha_prev * (1.0 + sig * alpha);
          zn[l] = zeta[l] * zeta_prev[l] * alpha_prev / den;
        }
        axpby(-alpha, q.p, 1.0, r.p);
        const double rr_new = nrm2(r.p);
        OVL_REQUIRE(std::isfinite(rr_new), OVL_E_NAN, "multi-shift CG: NaN in the residual");
        const double beta = rr_new / rr;
        for (int l = 0; l < n; ++l) {
          coef[4 * l + 3] = active[l] ? 1.0 : 0.0;
          if (!active[l]) continue;
          coef[4 * l] = alpha * zn[l] / zeta[l];
          coef[4 * l + 1] = zn[l];
          coef[4 * l + 2] = beta * (zn[l] / zeta[l]) * (zn[l] / zeta[l]);
        }
        OVL_HIP(hipMemcpyAsync(cf.p, coef.data(), sizeof(double) * 4 * n, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(shift_update_kernel, dim3((n16 + 255) / 256), dim3(256), 0, s, n16, n,
                           static_cast<const double2*>(r.p), static_cast<double2*>(X.p),
                           static_cast<double2*>(Pm.p), n16, static_cast<const double*>(cf.p));
        OVL_HIP(hipGetLastError());
        axpby(1.0, r.p, beta, p.p);  // p = r + beta p (synchronises: coef is free again)
        for (int l = 0; l < n; ++l) {
          if (!active[l]) continue;
          zeta_prev[l] = zeta[l];
          zeta[l] = zn[l];
          if (std::fabs(zn[l]) * std::sqrt(rr_new) <= tol * bn) {
            active[l] = 0;
            --nact;
          }
        }
        alpha_prev = alpha;
        beta_prev = beta;
        rr = rr_new;
        ++its;
      }
      stats->iterations = its;
      // pq = sum_l b_l x_l
      std::vector<double2> bc(n);
      for (int l = 0; l < n; ++l) bc[l] = make_double2(rat->b[l], 0.0);
      WsBuf bdev(sizeof(double2) * n, s);
      OVL_HIP(hipMemcpyAsync(bdev.p, bc.data(), sizeof(double2) * n, hipMemcpyHostToDevice, s));
      block_axpy(g, X.p, n, static_cast<const double2*>(bdev.p), pq.p, OVL_F64, 1, false, s);
      OVL_HIP(hipStreamSynchronize(s));
    } else {
      // ------------------------------------------------ double pass
      WsBuf v(v64, s), vp(v64, s), w(v64, s);
      const double bn = std::sqrt(bn2);
      std::vector<double> al, be, y;
      // pass 1: the Lanczos coefficients of Q^2 from v_1 = psi_h / ||psi_h||
      axpby(1.0 / bn, psih.p, 0.0, v.p);
      blas_zero(vp.p, v64, s);
      double beta = 0.0;
      for (;;) {
        if (static_cast<int>(al.size()) >= maxiter) {
          rc = OVL_W_NOT_CONVERGED;
          break;
        }
        qapply(t.p, v.p, nullptr, 0.0);
        qapply(w.p, t.p, nullptr, 0.0);
        if (beta != 0.0) axpby(-beta, vp.p, 1.0, w.p);
        const double a = dot_re(v.p, w.p);
        axpby(-a, v.p, 1.0, w.p);
        beta = std::sqrt(nrm2(w.p));
        OVL_REQUIRE(std::isfinite(a) && std::isfinite(beta), OVL_E_NAN, "double pass: NaN in the Lanczos recurrence");
        al.push_back(a);
        be.push_back(beta);
        y = tridiag_rational_e1(al, be, rat);
        if (beta == 0.0) break;
        if (y.size() >= 2) {
          // truncation error: the coupling to the next vector, summed as a
          // geometric series with the observed decay of the coefficients
          const double q = std::fabs(y[y.size() - 1]) / std::max(std::fabs(y[y.size() - 2]), 1e-300);
          const double tail = beta * std::fabs(y.back()) / std::max(1.0 - q, 1e-3);
          if (tail <= tol * std::fabs(y[0])) break;
        }
        std::swap(vp.p, v.p);  // v_prev <- v
        axpby(1.0 / beta, w.p, 0.0, v.p);
      }
      const int k = static_cast<int>(al.size());
      stats->iterations = k;
      // pass 2: the same recurrence again, summing y_j v_j
      axpby(1.0 / bn, psih.p, 0.0, v.p);
      blas_zero(vp.p, v64, s);
      axpby(y[0] * bn, v.p, 0.0, pq.p);
      for (int j = 1; j < k; ++j) {
        qapply(t.p, v.p, nullptr, 0.0);
        qapply(w.p, t.p, nullptr, 0.0);
        hipLaunchKernelGGL(lanczos_step_kernel, dim3((n16 + 255) / 256), dim3(256), 0, s, n16,
                           static_cast<double2*>(w.p), static_cast<double2*>(v.p), static_cast<double2*>(vp.p),
                           static_cast<double2*>(pq.p), al[j - 1], j >= 2 ? be[j - 2] : 0.0, 1.0 / be[j - 1],
                           y[j] * bn);
        OVL_HIP(hipGetLastError());
      }
      OVL_HIP(hipStreamSynchronize(s));
    }
    // out = Q pq (+ the low-mode part)
    if (lm)
      qapply(out, pq.p, wlow.p, 1.0);
    else
      qapply(out, pq.p, nullptr, 0.0);
    OVL_HIP(hipStreamSynchronize(s));
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (log_on())
      fprintf(stderr, "[ovl rational] %s, n = %d: %d iterations, %lld H_w applications, %.3f s\n",
              method == 0 ? "multi-shift CG" : "double pass", n, stats->iterations,
              static_cast<long long>(stats->hw_applies), stats->seconds);
    return rc;
  });
}

}  // extern "C"
