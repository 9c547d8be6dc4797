// Spectral set-up for the sign function (arXiv:1106.4964 Sec. V):
//
//  * ovl_hw_bound: Lanczos on H_w (FP64, full re-orthogonalisation) gives an
//    upper bound lam_max on |spectrum(H_w)| = max over the two extreme Ritz
//    pairs of |theta| + ||H_w y - theta y||; the normalisation Q = H_w/lam_max
//    must not exceed 1 in modulus.
//  * ovl_hw_eigs: the ell eigenpairs of H_w closest to zero.  The paper
//    runs implicitly restarted Arnoldi on a Chebyshev polynomial of H_w^2,
//    which has the same eigenvectors and a better separated spectrum
//    (Sec. V).  H_w is Hermitian, so here the Krylov method is thick-restart
//    Lanczos (full re-orthogonalisation) on B = T_d(Z), Z = (2 H_w^2 - a - b)
//    / (b - a), which maps |lambda|^2 in [a, b] into [-1, 1] and lifts the
//    wanted |lambda|^2 < a far above it.  The top Ritz vectors of B span the
//    wanted invariant subspace; Rayleigh-Ritz with H_w itself on that span
//    separates the +-lambda pairs B cannot tell apart and fixes the signs.
//    Stops when the ell pairs with smallest |theta| have
//    ||H_w v - theta v|| <= tol * lam_max.
//
// Dense m x m problems (Gram and Rayleigh-Ritz matrices, the Lanczos
// tridiagonal) are solved on the host by cyclic complex Jacobi rotations.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <numeric>

#include "ops.h"

namespace ovl {

using zc = std::complex<double>;

// Eigen-decomposition of a Hermitian n x n matrix A (column-major, A[i + n*j]).
// On exit w holds the eigenvalues in ascending order and V (column-major)
// the orthonormal eigenvectors.  Cyclic Jacobi: each rotation first turns
// A_pq real with a phase on column q, then zeroes it with a real rotation.
void host_heev(int n, std::vector<zc> A, std::vector<double>& w, std::vector<zc>& V) {
  V.assign(static_cast<size_t>(n) * n, zc(0.0, 0.0));
  for (int i = 0; i < n; ++i) V[i + static_cast<size_t>(n) * i] = 1.0;
  auto at = [&](int i, int j) -> zc& { return A[i + static_cast<size_t>(n) * j]; };
  double fro = 0.0;
  for (auto& v : A) fro += std::norm(v);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int q = 0; q < n; ++q)
      for (int p = 0; p < q; ++p) off += std::norm(at(p, q));
    if (off <= 1e-32 * fro || off == 0.0) break;
    for (int q = 1; q < n; ++q) {
      for (int p = 0; p < q; ++p) {
        const zc apq = at(p, q);
        const double c = std::abs(apq);
        if (c == 0.0 || c < 1e-300) continue;
        const zc u = apq / c;  // A_pq = c u
        const double app = at(p, p).real(), aqq = at(q, q).real();
        const double tau = (aqq - app) / (2.0 * c);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = t * cs;
        const zc ub = std::conj(u);
        // G = [[cs, sn], [-sn*ub, cs*ub]] on (p, q):  A <- G^H A G,  V <- V G
        for (int i = 0; i < n; ++i) {  // columns
          const zc aip = at(i, p), aiq = at(i, q);
          at(i, p) = cs * aip - sn * ub * aiq;
          at(i, q) = sn * aip + cs * ub * aiq;
        }
        for (int j = 0; j < n; ++j) {  // rows
          const zc apj = at(p, j), aqj = at(q, j);
          at(p, j) = cs * apj - sn * u * aqj;
          at(q, j) = sn * apj + cs * u * aqj;
        }
        at(p, q) = 0.0;
        at(q, p) = 0.0;
        at(p, p) = at(p, p).real();
        at(q, q) = at(q, q).real();
        for (int i = 0; i < n; ++i) {
          zc& vp = V[i + static_cast<size_t>(n) * p];
          zc& vq = V[i + static_cast<size_t>(n) * q];
          const zc a = vp, b = vq;
          vp = cs * a - sn * ub * b;
          vq = sn * a + cs * ub * b;
        }
      }
    }
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::vector<double> d(n);
  for (int i = 0; i < n; ++i) d[i] = at(i, i).real();
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
  w.resize(n);
  std::vector<zc> Vs(static_cast<size_t>(n) * n);
  for (int k = 0; k < n; ++k) {
    w[k] = d[order[k]];
    for (int i = 0; i < n; ++i) Vs[i + static_cast<size_t>(n) * k] = V[i + static_cast<size_t>(n) * order[k]];
  }
  V.swap(Vs);
}

namespace {

struct Hw {
  const ovl_gauge* u;
  double rho;
  hipStream_t s;
  size_t v64;
  const void* links;
  int recon;
  int64_t applies = 0;

  // out = scale * H_w in + sum_j c_j v_j   (batch of R FP64 vectors)
  void apply(void* out, const void* in, int R, double scale = 1.0, const void* v0 = nullptr, double c0 = 0.0,
             const void* v1 = nullptr, double c1 = 0.0) {
    StencilArgs A{};
    A.g = u->geom.geo;
    A.out = out;
    A.in = in;
    A.links = links;
    A.a = scale * (4.0 - rho);
    A.b = -0.5 * scale;
    A.g5 = 1;
    A.par0 = 0;
    A.npar = 2;
    A.vstride = v64;
    A.nv = 0;
    if (v0) {
      A.v[A.nv] = v0;
      A.cv[A.nv++] = c0;
    }
    if (v1) {
      A.v[A.nv] = v1;
      A.cv[A.nv++] = c1;
    }
    launch_stencil(A, OVL_F64, recon, R, s);
    applies += R;
  }
};

struct DevMem {
  void* p = nullptr;
  size_t n = 0;
  explicit DevMem(size_t bytes) : n(bytes) {
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(OVL_E_NOMEM, "eigensolver: device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    mem_track(static_cast<int64_t>(n));
  }
  ~DevMem() {
    if (p) {
      (void)hipFree(p);
      mem_track(-static_cast<int64_t>(n));
    }
  }
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
};

char* vec(void* base, size_t v64, int i) { return static_cast<char*>(base) + static_cast<size_t>(i) * v64; }

// G = V^dag W for m basis vectors V and k vectors W (host, column-major m x k).
std::vector<zc> gram(const ovl_geom* g, const void* V, int m, const void* W, int k, size_t v64, hipStream_t s) {
  std::vector<zc> G(static_cast<size_t>(m) * k);
  WsBuf cb(static_cast<size_t>(m) * OVL_MAX_RHS * sizeof(double2), s);
  std::vector<double2> host(static_cast<size_t>(m) * OVL_MAX_RHS);
  for (int c0 = 0; c0 < k; c0 += OVL_MAX_RHS) {
    const int R = std::min(OVL_MAX_RHS, k - c0);
    block_dot(g, V, m, vec(const_cast<void*>(W), v64, c0), OVL_F64, R, static_cast<double2*>(cb.p), s);
    OVL_HIP(hipMemcpyAsync(host.data(), cb.p, sizeof(double2) * m * R, hipMemcpyDeviceToHost, s));
    OVL_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < m; ++i)
      for (int r = 0; r < R; ++r) G[i + static_cast<size_t>(m) * (c0 + r)] = zc(host[i * R + r].x, host[i * R + r].y);
  }
  return G;
}

// Y = V M for m basis vectors and an m x k host matrix M (column-major).
void rotate(const ovl_geom* g, const void* V, int m, const std::vector<zc>& M, int k, void* Y, size_t v64,
            hipStream_t s) {
  WsBuf kb(static_cast<size_t>(m) * OVL_MAX_RHS * sizeof(double2), s);
  std::vector<double2> host(static_cast<size_t>(m) * OVL_MAX_RHS);
  for (int c0 = 0; c0 < k; c0 += OVL_MAX_RHS) {
    const int R = std::min(OVL_MAX_RHS, k - c0);
    for (int i = 0; i < m; ++i)
      for (int r = 0; r < R; ++r) {
        const zc v = M[i + static_cast<size_t>(m) * (c0 + r)];
        host[i * R + r] = make_double2(v.real(), v.imag());
      }
    OVL_HIP(hipMemcpyAsync(kb.p, host.data(), sizeof(double2) * m * R, hipMemcpyHostToDevice, s));
    block_axpy(g, V, m, static_cast<const double2*>(kb.p), vec(Y, v64, c0), OVL_F64, R, false, s);
    OVL_HIP(hipStreamSynchronize(s));  // host staging buffer is reused
  }
}

}  // namespace
}  // namespace ovl

using namespace ovl;

extern "C" {

int ovl_host_heev(int n, const double* A, double* w, double* V) {
  return guard([&] {
    OVL_REQUIRE(n >= 1 && A && w && V, OVL_E_ARG, "null argument");
    std::vector<zc> a(static_cast<size_t>(n) * n);
    for (size_t k = 0; k < a.size(); ++k) a[k] = zc(A[2 * k], A[2 * k + 1]);
    std::vector<double> ww;
    std::vector<zc> vv;
    host_heev(n, a, ww, vv);
    for (int i = 0; i < n; ++i) w[i] = ww[i];
    for (size_t k = 0; k < vv.size(); ++k) {
      V[2 * k] = vv[k].real();
      V[2 * k + 1] = vv[k].imag();
    }
    return OVL_OK;
  });
}

int ovl_hw_bound(const ovl_gauge* u, double rho, const void* v0, int steps, double* lam_max, double* theta_min,
                 double* theta_max, ovl_stream_t st) {
  return guard([&] {
    OVL_REQUIRE(u && v0 && lam_max, OVL_E_ARG, "null argument");
    OVL_REQUIRE(steps >= 2 && steps <= 1000, OVL_E_ARG, "steps out of range");
    hipStream_t s = static_cast<hipStream_t>(st);
    const ovl_geom* g = &u->geom;
    Hw H{u, rho, s, spinor_vec_bytes(g, OVL_F64), nullptr, 0};
    H.links = gauge_links(u, OVL_F64, &H.recon);
    const size_t v64 = H.v64;
    DevMem Q(v64 * (steps + 1));
    WsBuf w(v64, s), sc(4 * sizeof(double), s), cb(sizeof(double2) * (steps + 1), s);
    // q0 = v0 / ||v0||
    auto norm = [&](const void* x) {
      blas_norm2(OVL_F64, v64 / 16, x, 1, v64, static_cast<double*>(sc.p), s);
      double h[2];
      OVL_HIP(hipMemcpyAsync(h, sc.p, sizeof(h), hipMemcpyDeviceToHost, s));
      OVL_HIP(hipStreamSynchronize(s));
      return std::sqrt(h[0]);
    };
    auto scale_into = [&](void* dst, const void* src, double a) {
      double h[2] = {a, 0.0};
      OVL_HIP(hipMemcpyAsync(sc.p, h, sizeof(h), hipMemcpyHostToDevice, s));
      blas_axpby(OVL_F64, src, static_cast<double*>(sc.p), OVL_F64, dst, nullptr, g->N, 1, s);
      OVL_HIP(hipStreamSynchronize(s));
    };
    const double n0 = norm(v0);
    OVL_REQUIRE(n0 > 0.0 && std::isfinite(n0), OVL_E_ARG, "start vector is zero or not finite");
    scale_into(vec(Q.p, v64, 0), v0, 1.0 / n0);
    std::vector<double> alpha, beta;
    std::vector<double2> hc(steps + 1);
    for (int j = 0; j < steps; ++j) {
      H.apply(w.p, vec(Q.p, v64, j), 1);
      // full re-orthogonalisation (twice): w -= Q (Q^dag w); alpha_j = (q_j^dag w) of the first pass
      double aj = 0.0;
      for (int pass = 0; pass < 2; ++pass) {
        block_dot(g, Q.p, j + 1, w.p, OVL_F64, 1, static_cast<double2*>(cb.p), s);
        OVL_HIP(hipMemcpyAsync(hc.data(), cb.p, sizeof(double2) * (j + 1), hipMemcpyDeviceToHost, s));
        OVL_HIP(hipStreamSynchronize(s));
        if (pass == 0) aj = hc[j].x;
        else aj += hc[j].x;
        for (int i = 0; i <= j; ++i) hc[i] = make_double2(-hc[i].x, -hc[i].y);
        OVL_HIP(hipMemcpyAsync(cb.p, hc.data(), sizeof(double2) * (j + 1), hipMemcpyHostToDevice, s));
        block_axpy(g, Q.p, j + 1, static_cast<const double2*>(cb.p), w.p, OVL_F64, 1, true, s);
        OVL_HIP(hipStreamSynchronize(s));
      }
      alpha.push_back(aj);
      const double bj = norm(w.p);
      beta.push_back(bj);
      if (bj < 1e-14 * std::fabs(aj) || j == steps - 1) break;
      scale_into(vec(Q.p, v64, j + 1), w.p, 1.0 / bj);
    }
    const int k = static_cast<int>(alpha.size());
    std::vector<zc> T(static_cast<size_t>(k) * k, zc(0.0, 0.0));
    for (int i = 0; i < k; ++i) {
      T[i + static_cast<size_t>(k) * i] = alpha[i];
      if (i + 1 < k) {
        T[i + 1 + static_cast<size_t>(k) * i] = beta[i];
        T[i + static_cast<size_t>(k) * (i + 1)] = beta[i];
      }
    }
    std::vector<double> th;
    std::vector<zc> S;
    host_heev(k, T, th, S);
    const double bk = beta[k - 1];
    const double r_lo = std::fabs(bk) * std::abs(S[(k - 1) + static_cast<size_t>(k) * 0]);
    const double r_hi = std::fabs(bk) * std::abs(S[(k - 1) + static_cast<size_t>(k) * (k - 1)]);
    *lam_max = std::max(std::fabs(th[0]) + r_lo, std::fabs(th[k - 1]) + r_hi);
    if (theta_min) *theta_min = th[0];
    if (theta_max) *theta_max = th[k - 1];
    return OVL_OK;
  });
}

int ovl_hw_eigs(const ovl_gauge* u, double rho, int ell, int m, void* V, double* lambda, double lam_max, double tol,
                int max_iter, int degree, ovl_eig_stats* stats, ovl_stream_t st) {
  return guard([&] {
    OVL_REQUIRE(u && V && lambda && stats, OVL_E_ARG, "null argument");
    OVL_REQUIRE(lam_max > 0.0 && tol > 0.0 && max_iter >= 1 && degree >= 1, OVL_E_ARG, "bad eigensolver parameter");
    const int want = ell + std::max(8, ell / 10);  // cushion: a +-lambda pair may straddle the cut
    OVL_REQUIRE(ell >= 1 && m >= want, OVL_E_ARG, "need m >= ell + max(8, ell/10) vectors in V");
    OVL_REQUIRE(want + 40 <= 512, OVL_E_ARG, "at most 429 eigenpairs (the Lanczos basis holds 512 vectors)");
    // Lanczos basis: 2 want (at least want + 40, at most 512) vectors, cut
    // back toward want + 40 while the basis and its work vectors would take
    // more than 90% of the free device memory (large volumes with many modes)
    int K = std::min(512, std::max(2 * want, want + 40));
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = static_cast<hipStream_t>(st);
    const ovl_geom* g = &u->geom;
    {
      size_t fr = 0, tot = 0;
      OVL_HIP(hipMemGetInfo(&fr, &tot));
      const size_t vb = spinor_vec_bytes(g, OVL_F64);
      auto need = [&](int k) { return vb * (k + 5) + sizeof(double2) * static_cast<size_t>(k) * k; };
      while (K > want + 40 && static_cast<double>(need(K)) > 0.9 * static_cast<double>(fr)) K -= 8;
      K = std::max(K, std::min(512, want + 40));
    }
    const int keep = want + (K - want) / 2;  // thick-restart size
    Hw H{u, rho, s, spinor_vec_bytes(g, OVL_F64), nullptr, 0};
    H.links = gauge_links(u, OVL_F64, &H.recon);
    const size_t v64 = H.v64;
    DevMem Q(v64 * (K + 1));
    DevMem ya(v64), yb(v64), tt(v64), w(v64);
    WsBuf sc(2 * sizeof(double), s), cb(sizeof(double2) * (K + 1), s);
    DevMem Sdev(sizeof(double2) * static_cast<size_t>(K) * K);
    *stats = ovl_eig_stats{};

    auto norm = [&](const void* x) {
      blas_norm2(OVL_F64, v64 / 16, x, 1, v64, static_cast<double*>(sc.p), s);
      double h[2];
      OVL_HIP(hipMemcpyAsync(h, sc.p, sizeof(h), hipMemcpyDeviceToHost, s));
      OVL_HIP(hipStreamSynchronize(s));
      return std::sqrt(h[0]);
    };
    auto scale_into = [&](void* dst, const void* src, double a) {
      double h[2] = {a, 0.0};
      OVL_HIP(hipMemcpyAsync(sc.p, h, sizeof(h), hipMemcpyHostToDevice, s));
      blas_axpby(OVL_F64, src, static_cast<double*>(sc.p), OVL_F64, dst, nullptr, g->N, 1, s);
      OVL_HIP(hipStreamSynchronize(s));
    };
    auto upload_S = [&](const std::vector<zc>& S, int rows, int cols) {
      std::vector<double2> h(static_cast<size_t>(rows) * cols);
      for (size_t i = 0; i < h.size(); ++i) h[i] = make_double2(S[i].real(), S[i].imag());
      OVL_HIP(hipMemcpyAsync(Sdev.p, h.data(), h.size() * sizeof(double2), hipMemcpyHostToDevice, s));
      OVL_HIP(hipStreamSynchronize(s));
    };

    double cut = 0.15 * lam_max;  // lower edge of the damped band
    const double b2 = lam_max * lam_max;
    // B x = T_degree(Z) x, three-term recurrence, result in `out`
    auto applyB = [&](void* out, const void* x, double a2) {
      const double e = 0.5 * (b2 - a2), cc = 0.5 * (b2 + a2);
      H.apply(tt.p, x, 1);
      if (degree == 1) {
        H.apply(out, tt.p, 1, 1.0 / e, x, -cc / e);
        return;
      }
      H.apply(ya.p, tt.p, 1, 1.0 / e, x, -cc / e);  // y1
      const void* yprev = x;
      void* ycur = ya.p;
      for (int j = 1; j < degree; ++j) {
        void* dst = (j == degree - 1) ? out : (yprev == x ? yb.p : const_cast<void*>(yprev));
        H.apply(tt.p, ycur, 1);
        H.apply(dst, tt.p, 1, 2.0 / e, ycur, -2.0 * cc / e, yprev, -1.0);
        yprev = ycur;
        ycur = dst;
      }
    };

    // q_0 from the caller's start vector V[:, 0]
    {
      const double n0 = norm(V);
      OVL_REQUIRE(n0 > 0.0 && std::isfinite(n0), OVL_E_ARG, "start vector V[:,0] is zero or not finite");
      scale_into(vec(Q.p, v64, 0), V, 1.0 / n0);
    }
    std::vector<zc> T(static_cast<size_t>(K + 1) * (K + 1), zc(0.0, 0.0));
    auto Tat = [&](int i, int j) -> zc& { return T[i + static_cast<size_t>(K + 1) * j]; };
    std::vector<double2> hc(K + 1), hc2(K + 1);
    std::vector<double> theta(want), res(ell, INFINITY);
    int cur = 0;
    for (int cycle = 0;; ++cycle) {
      const double a2 = cut * cut;
      for (int j = cur; j < K; ++j) {
        applyB(w.p, vec(Q.p, v64, j), a2);
        // w -= Q (Q^dag w), twice; the coefficients of both passes form column j of T
        for (int i = 0; i <= j; ++i) hc2[i] = make_double2(0.0, 0.0);
        for (int pass = 0; pass < 2; ++pass) {
          block_dot(g, Q.p, j + 1, w.p, OVL_F64, 1, static_cast<double2*>(cb.p), s);
          OVL_HIP(hipMemcpyAsync(hc.data(), cb.p, sizeof(double2) * (j + 1), hipMemcpyDeviceToHost, s));
          OVL_HIP(hipStreamSynchronize(s));
          for (int i = 0; i <= j; ++i) {
            hc2[i] = make_double2(hc2[i].x + hc[i].x, hc2[i].y + hc[i].y);
            hc[i] = make_double2(-hc[i].x, -hc[i].y);
          }
          OVL_HIP(hipMemcpyAsync(cb.p, hc.data(), sizeof(double2) * (j + 1), hipMemcpyHostToDevice, s));
          block_axpy(g, Q.p, j + 1, static_cast<const double2*>(cb.p), w.p, OVL_F64, 1, true, s);
          OVL_HIP(hipStreamSynchronize(s));
        }
        for (int i = 0; i <= j; ++i) Tat(i, j) = zc(hc2[i].x, hc2[i].y);
        const double beta = norm(w.p);
        OVL_REQUIRE(std::isfinite(beta), OVL_E_NAN, "eigensolver: NaN in the Lanczos recurrence");
        Tat(j + 1, j) = beta;
        if (beta == 0.0) throw Error(OVL_E_BREAKDOWN, "eigensolver: invariant subspace found before K steps");
        scale_into(vec(Q.p, v64, j + 1), w.p, 1.0 / beta);
      }
      // Ritz pairs of B, largest first
      std::vector<zc> Tk(static_cast<size_t>(K) * K);
      for (int j = 0; j < K; ++j)
        for (int i = 0; i < K; ++i)
          Tk[i + static_cast<size_t>(K) * j] = 0.5 * (Tat(i, j) + std::conj(Tat(j, i)));
      std::vector<double> th;
      std::vector<zc> S;
      host_heev(K, Tk, th, S);
      std::reverse(th.begin(), th.end());
      std::vector<zc> Sd(static_cast<size_t>(K) * K);
      for (int c = 0; c < K; ++c)
        for (int i = 0; i < K; ++i) Sd[i + static_cast<size_t>(K) * c] = S[i + static_cast<size_t>(K) * (K - 1 - c)];
      const double betaK = Tat(K, K - 1).real();
      // the wanted block must stand clear of the damped band [-1, 1]
      if (th[want - 1] < 1.5 && cycle < max_iter) {
        cut *= 1.4;
        if (log_on()) fprintf(stderr, "[ovl eigs] cycle %d (basis %d): widening the damped band\n", cycle, K);
        // restart from the sum of the current top Ritz vectors
        upload_S(Sd, K, K);
        block_rotate_inplace(g, Q.p, K, static_cast<const double2*>(Sdev.p), 1, s);
        const double nq = norm(Q.p);
        scale_into(vec(Q.p, v64, 0), Q.p, 1.0 / nq);
        cur = 0;
        std::fill(T.begin(), T.end(), zc(0.0, 0.0));
        stats->iterations = cycle + 1;
        continue;
      }
      // span of the top `want` Ritz vectors -> V, then Rayleigh-Ritz with H_w
      {
        std::vector<zc> Sw(Sd.begin(), Sd.begin() + static_cast<size_t>(K) * want);
        rotate(g, Q.p, K, Sw, want, V, v64, s);
      }
      std::vector<zc> Hs(static_cast<size_t>(want) * want);
      for (int c0 = 0; c0 < want; c0 += OVL_MAX_RHS) {
        const int R = std::min(OVL_MAX_RHS, want - c0);
        for (int r = 0; r < R; ++r) {
          H.apply(w.p, vec(V, v64, c0 + r), 1);
          std::vector<zc> col = gram(g, V, want, w.p, 1, v64, s);
          for (int i = 0; i < want; ++i) Hs[i + static_cast<size_t>(want) * (c0 + r)] = col[i];
        }
      }
      for (int i = 0; i < want; ++i)
        for (int j = 0; j <= i; ++j) {
          const zc a = 0.5 * (Hs[i + static_cast<size_t>(want) * j] + std::conj(Hs[j + static_cast<size_t>(want) * i]));
          Hs[i + static_cast<size_t>(want) * j] = a;
          Hs[j + static_cast<size_t>(want) * i] = std::conj(a);
        }
      std::vector<double> lh;
      std::vector<zc> SH;
      host_heev(want, Hs, lh, SH);
      std::vector<int> ord(want);
      std::iota(ord.begin(), ord.end(), 0);
      std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
        return std::fabs(lh[x]) < std::fabs(lh[y]) || (std::fabs(lh[x]) == std::fabs(lh[y]) && lh[x] < lh[y]);
      });
      std::vector<zc> So(static_cast<size_t>(want) * want);
      for (int c = 0; c < want; ++c) {
        theta[c] = lh[ord[c]];
        for (int i = 0; i < want; ++i) So[i + static_cast<size_t>(want) * c] = SH[i + static_cast<size_t>(want) * ord[c]];
      }
      upload_S(So, want, want);
      block_rotate_inplace(g, V, want, static_cast<const double2*>(Sdev.p), want, s);
      double worst = 0.0;
      for (int i = 0; i < ell; ++i) {
        H.apply(w.p, vec(V, v64, i), 1, 1.0, vec(V, v64, i), -theta[i]);
        res[i] = norm(w.p);
        worst = std::max(worst, res[i]);
      }
      stats->iterations = cycle + 1;
      stats->max_residual = worst;
      if (log_on())
        fprintf(stderr, "[ovl eigs] cycle %d (basis %d): max residual %.3e, target %.3e\n", cycle, K, worst,
                tol * lam_max);
      if (worst <= tol * lam_max || cycle + 1 >= max_iter) break;
      // thick restart: keep the top `keep` Ritz vectors of B and the residual direction
      upload_S(Sd, K, K);
      block_rotate_inplace(g, Q.p, K, static_cast<const double2*>(Sdev.p), keep, s);
      OVL_HIP(hipMemcpyAsync(vec(Q.p, v64, keep), vec(Q.p, v64, K), v64, hipMemcpyDeviceToDevice, s));
      std::fill(T.begin(), T.end(), zc(0.0, 0.0));
      for (int i = 0; i < keep; ++i) {
        Tat(i, i) = th[i];
        const zc c = betaK * Sd[(K - 1) + static_cast<size_t>(K) * i];
        Tat(keep, i) = c;
        Tat(i, keep) = std::conj(c);
      }
      cur = keep;
    }
    for (int i = 0; i < ell; ++i) lambda[i] = theta[i];
    OVL_HIP(hipStreamSynchronize(s));
    stats->hw_applies = H.applies;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return stats->max_residual <= tol * lam_max ? OVL_OK : OVL_W_NOT_CONVERGED;
  });
}

}  // extern "C"
