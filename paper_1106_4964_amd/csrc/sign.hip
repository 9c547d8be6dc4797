// Polynomial sign function with low-mode projection, and the overlap
// operator (arXiv:1106.4964 Sec. II eq. 3-8, Sec. V).
//
//   sign(H_w) psi = sum_i sign(lambda_i) (eta_i^dag psi) eta_i + Q P(Q^2) psi_h,
//   psi_h = psi - sum_i (eta_i^dag psi) eta_i,   Q = H_w / lam_max,
//   P(x) = sum_k c_k T_k(y),  y = (2x - 1 - eps)/(1 - eps), the optimal
//   polynomial of order n (eq. 4; coefficients by the Remez exchange below),
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
// The points go through the Clenshaw recursion 16 at a time (independent
// lanes the compiler vectorises); a NaN anywhere gives INFINITY.
double sign_delta(const std::vector<double>& c, double eps, int npts = 400000) {
  constexpr int B = 16;
  const int half = npts / 2, rest = npts - half;
  const double pi = 3.14159265358979323846;
  const int nc = static_cast<int>(c.size());
  auto point = [&](int i) {
    if (i < half) return half == 1 ? eps : eps + (1.0 - eps) * i / (half - 1);
    const int j = i - half;
    const double th = rest == 1 ? 0.0 : pi * j / (rest - 1);
    return 0.5 * ((1.0 - eps) * std::cos(th) + 1.0 + eps);
  };
  double worst = 0.0;
  bool nan = false;
  for (int i0 = 0; i0 < npts; i0 += B) {
    const int cnt = std::min(B, npts - i0);
    double x[B], y[B], b1[B], b2[B];
    for (int l = 0; l < B; ++l) {
      x[l] = point(i0 + std::min(l, cnt - 1));
      y[l] = (2.0 * x[l] - 1.0 - eps) / (1.0 - eps);
      b1[l] = 0.0;
      b2[l] = 0.0;
    }
    for (int k = nc - 1; k >= 1; --k) {
      const double ck = c[k];
      for (int l = 0; l < B; ++l) {
        const double b = ck + 2.0 * y[l] * b1[l] - b2[l];
        b2[l] = b1[l];
        b1[l] = b;
      }
    }
    for (int l = 0; l < cnt; ++l) {
      const double d = std::fabs(1.0 - std::sqrt(x[l]) * (c[0] + y[l] * b1[l] - b2[l]));
      if (d != d) nan = true;
      else worst = std::max(worst, d);
    }
  }
  return nan ? INFINITY : worst;
}

// ------------------------------------------------------ optimal polynomial
// P of order n minimising delta = max |1 - sqrt(x) P(x)| over [eps, 1] (the
// optimal approximation of eq. 4; Fig. 2 prints delta = 0.1 at n = 13,
// sqrt(eps) ~ 0.06).  Remez exchange on the relative error, P kept as
// Chebyshev coefficients in y: on a reference r_0 < ... < r_{n+1} the linear
// system sum_k c_k T_k(y(r_i)) + (-1)^i E / sqrt(r_i) = 1 / sqrt(r_i)
// levels the error to (-1)^i E; the error then has one zero between
// consecutive reference points (found by bisection) and the next reference
// is the peak of |error| between consecutive zeros, the ends eps and 1
// included (golden-section search).  The start is the Chebyshev
// interpolant, whose error vanishes at its n+1 nodes.  Kept instead of the
// exchange: the interpolant itself when its delta is at the level of FP64
// rounding (<= 1e-12, nothing left to level) or the order is above 400
// (the dense (n+2)^2 system), and whenever the exchange ends worse.
namespace {

constexpr double kRoundingDelta = 1e-12;
constexpr int kMinimaxMaxOrder = 400;

double cheb_value(const std::vector<double>& c, double y) {
  double b1 = 0.0, b2 = 0.0;
  for (int k = static_cast<int>(c.size()) - 1; k >= 1; --k) {
    const double b = c[k] + 2.0 * y * b1 - b2;
    b2 = b1;
    b1 = b;
  }
  return c[0] + y * b1 - b2;
}

// 1 - sqrt(x) P(x)
double rel_error(const std::vector<double>& c, double eps, double x) {
  return 1.0 - std::sqrt(x) * cheb_value(c, (2.0 * x - 1.0 - eps) / (1.0 - eps));
}

// Solves the m x m row-major system in place (Gaussian elimination with
// partial pivoting); false when a pivot vanishes.
bool dense_solve(std::vector<double>& a, std::vector<double>& rhs, int m) {
  for (int col = 0; col < m; ++col) {
    int piv = col;
    for (int r = col + 1; r < m; ++r)
      if (std::fabs(a[static_cast<size_t>(r) * m + col]) > std::fabs(a[static_cast<size_t>(piv) * m + col])) piv = r;
    if (a[static_cast<size_t>(piv) * m + col] == 0.0) return false;
    if (piv != col) {
      for (int k = 0; k < m; ++k) std::swap(a[static_cast<size_t>(col) * m + k], a[static_cast<size_t>(piv) * m + k]);
      std::swap(rhs[col], rhs[piv]);
    }
    const double d = a[static_cast<size_t>(col) * m + col];
    for (int r = col + 1; r < m; ++r) {
      const double f = a[static_cast<size_t>(r) * m + col] / d;
      if (f == 0.0) continue;
      for (int k = col; k < m; ++k) a[static_cast<size_t>(r) * m + k] -= f * a[static_cast<size_t>(col) * m + k];
      rhs[r] -= f * rhs[col];
    }
  }
  for (int r = m - 1; r >= 0; --r) {
    double v = rhs[r];
    for (int k = r + 1; k < m; ++k) v -= a[static_cast<size_t>(r) * m + k] * rhs[k];
    rhs[r] = v / a[static_cast<size_t>(r) * m + r];
  }
  return true;
}

// Point of largest |error| in [a, b]: golden-section search, then the
// better of its result and the two ends.
double peak_of(const std::vector<double>& c, double eps, double a, double b) {
  const double g = 0.5 * (std::sqrt(5.0) - 1.0);
  double lo = a, hi = b;
  for (int it = 0; it < 64; ++it) {
    const double x1 = hi - g * (hi - lo), x2 = lo + g * (hi - lo);
    if (std::fabs(rel_error(c, eps, x1)) > std::fabs(rel_error(c, eps, x2))) hi = x2;
    else lo = x1;
  }
  double best = a, fb = std::fabs(rel_error(c, eps, a));
  for (double x : {0.5 * (lo + hi), b}) {
    const double f = std::fabs(rel_error(c, eps, x));
    if (f > fb) {
      fb = f;
      best = x;
    }
  }
  return best;
}

// A zero of the error in [a, b], the error differing in sign at the ends.
double zero_of(const std::vector<double>& c, double eps, double a, double b) {
  double fa = rel_error(c, eps, a);
  for (int it = 0; it < 60; ++it) {
    const double m = 0.5 * (a + b), fm = rel_error(c, eps, m);
    if ((fm < 0.0) != (fa < 0.0)) {
      b = m;
    } else {
      a = m;
      fa = fm;
    }
  }
  return 0.5 * (a + b);
}

}  // namespace

// The optimal coefficients of order n; *delta receives their measured delta.
std::vector<double> minimax_coeffs(double eps, int n, double* delta) {
  const std::vector<double> c0 = cheb_coeffs(eps, n);
  const double d0 = sign_delta(c0, eps);
  *delta = d0;
  if (d0 <= kRoundingDelta || n > kMinimaxMaxOrder) return c0;
  const double pi = 3.14159265358979323846;
  const int m = n + 2;
  std::vector<double> edge(n + 3);
  edge[0] = eps;
  edge[n + 2] = 1.0;
  for (int j = 0; j <= n; ++j)  // the interpolant's nodes, ascending in x
    edge[n + 1 - j] = 0.5 * ((1.0 - eps) * std::cos(pi * (j + 0.5) / (n + 1)) + 1.0 + eps);
  std::vector<double> ref(m);
  for (int i = 0; i < m; ++i) ref[i] = peak_of(c0, eps, edge[i], edge[i + 1]);
  std::vector<double> c = c0, a(static_cast<size_t>(m) * m), rhs(m);
  double best_gap = INFINITY;
  int stall = 0;
  for (int it = 0; it < 60; ++it) {
    for (int i = 0; i < m; ++i) {
      const double y = (2.0 * ref[i] - 1.0 - eps) / (1.0 - eps);
      double* row = &a[static_cast<size_t>(i) * m];
      row[0] = 1.0;
      if (n >= 1) row[1] = y;
      for (int k = 2; k <= n; ++k) row[k] = 2.0 * y * row[k - 1] - row[k - 2];
      row[n + 1] = ((i & 1) ? -1.0 : 1.0) / std::sqrt(ref[i]);
      rhs[i] = 1.0 / std::sqrt(ref[i]);
    }
    if (!dense_solve(a, rhs, m)) break;
    std::vector<double> cn(rhs.begin(), rhs.begin() + n + 1);
    const double E = std::fabs(rhs[n + 1]);
    if (!(E > 0.0) || !std::isfinite(E)) break;
    c = cn;
    edge[0] = eps;
    edge[n + 2] = 1.0;
    for (int i = 0; i + 1 < m; ++i) edge[i + 1] = zero_of(c, eps, ref[i], ref[i + 1]);
    double top = 0.0;
    for (int i = 0; i < m; ++i) {
      ref[i] = peak_of(c, eps, edge[i], edge[i + 1]);
      top = std::max(top, std::fabs(rel_error(c, eps, ref[i])));
    }
    const double gap = top / E - 1.0;
    if (gap < 1e-10) break;
    if (gap < 0.999 * best_gap) {
      best_gap = gap;
      stall = 0;
    } else if (++stall >= 3) {
      break;  // e is at the level of rounding: no further levelling
    }
  }
  const double d = sign_delta(c, eps);
  if (d >= d0) return c0;
  *delta = d;
  return c;
}

// Smallest n with measured delta <= target, searched from the order law
// delta = 0.41 exp(-2.1 n sqrt(eps)) (eq. 11): bracket, then bisect.
int interp_order(double eps, double target) {
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

// Smallest n whose optimal polynomial has measured delta <= target: the
// optimal delta is below the interpolant's at every n and falls with n, so
// the search starts at the interpolant's order and steps down.  Returns the
// coefficients of that order and their measured delta.
std::vector<double> sign_search(double eps, double target, double* delta) {
  int n = interp_order(eps, target);
  std::vector<double> c = minimax_coeffs(eps, n, delta);
  while (n > 1) {
    double d;
    std::vector<double> lower = minimax_coeffs(eps, n - 1, &d);
    if (d > target) break;
    c.swap(lower);
    *delta = d;
    --n;
  }
  return c;
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

namespace {
// mode: 0 = sign(H_w) in, 1 = ap in + am gamma5 sign(H_w) in,
//       2 = ap in + am sign(H_w) gamma5 in.
void overlap_driver(void* out, const void* in, const ovl_gauge* u, double rho, double ap, double am,
                    const ovl_sign* sg, const ovl_lowmodes* lm, int mode, int prec, int nrhs, hipStream_t s) {
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
}  // namespace

void overlap_apply(void* out, const void* in, const ovl_gauge* u, double rho, double m, const ovl_sign* sg,
                   const ovl_lowmodes* lm, int mode, int prec, int nrhs, hipStream_t s) {
  overlap_driver(out, in, u, rho, rho + 0.5 * m, rho - 0.5 * m, sg, lm, mode, prec, nrhs, s);
}

void overlap_combine(void* out, const void* in, const ovl_gauge* u, double rho, double ap, double am,
                     const ovl_sign* sg, const ovl_lowmodes* lm, int prec, int nrhs, hipStream_t s) {
  overlap_driver(out, in, u, rho, ap, am, sg, lm, 1, prec, nrhs, s);
}

void overlap_combine_dag(void* out, const void* in, const ovl_gauge* u, double rho, double ap, double am,
                         const ovl_sign* sg, const ovl_lowmodes* lm, int prec, int nrhs, hipStream_t s) {
  overlap_driver(out, in, u, rho, ap, am, sg, lm, 2, prec, nrhs, s);
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
    double measured = 0.0;
    std::vector<double> c = n > 0 ? minimax_coeffs(eps, n, &measured) : sign_search(eps, delta, &measured);
    ovl_sign* sg = new ovl_sign;
    sg->lam_max = lam_max;
    sg->eps = eps;
    sg->c = std::move(c);
    sg->delta = measured;
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

int ovl_lowmodes_project_noalloc(const ovl_lowmodes* lm, const void* in, void* psi_h, void* w, ovl_prec prec,
                                 int nrhs, ovl_stream_t s) {
  return guard([&] {
    OVL_REQUIRE(lm && in && psi_h && w, OVL_E_ARG, "null argument");
    check_prec(prec);
    check_nrhs(nrhs);
    OVL_REQUIRE(lm->ell > 0, OVL_E_ARG, "no low modes");
    OVL_REQUIRE(in != psi_h && in != w && psi_h != w, OVL_E_ALIAS, "projection outputs must not alias");
    lowmode_project_static(lm, in, psi_h, w, prec, nrhs, static_cast<hipStream_t>(s));
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
