// Low eigenpairs of the massless overlap operator from one chiral sector,
// and the deflation handle (arXiv:1106.4964 Sec. II eq. 9, Sec. V).
//
// D = 1 + gamma5 eps with eps = sign(H_w) (eq. 3).  gamma5 D = gamma5 + eps is
// Hermitian; on the chiral sector s (P_s = (1 + s gamma5)/2, spins 0-1 for
// s = +1, 2-3 for s = -1 in the chiral basis) its eigenvectors are those of
// K_s = s P_s eps P_s, whose eigenvalues k lie in [-1, 1].  The paper
// computes the overlap eigenvectors this way (Sec. V).  An eigenvector v of
// K_s gives, with w = P_{-s} eps v, sn = ||w|| = sqrt(1 - k^2) and u = w / sn,
// the invariant plane span(v, u) on which D has the eigenpairs
//     xi_+- = (v +- i u) / sqrt(2),   d_+- = 1 + k +- i s sn,
// and |d|^2 = 2 (1 + k): the modes closest to zero are the lowest k.  A real
// mode (sn = 0) gives d = 1 + k and xi = v.
//
// Krylov method: thick-restart Lanczos on K_s (FP64, full
// re-orthogonalisation, each matvec one sign application of the polynomial
// approximation with the low modes of H_w projected exactly, eq. 7), Ritz
// residuals from the Lanczos relation, the final ones recomputed from the
// same sign application that gives u.  The basis is kept as chiral
// half-vectors (the 6 components of chirality s per site), half the memory
// and half the re-orthogonalisation traffic of full spinors; a matvec
// expands its input into a full vector, applies the sign, and keeps the
// sector rows of the result.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>

#include "ops.h"

namespace ovl {

using zc = std::complex<double>;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  explicit DevBuf(size_t bytes) : n(bytes) {
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(OVL_E_NOMEM, "overlap eigensolver: device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    mem_track(static_cast<int64_t>(n));
  }
  ~DevBuf() {
    if (p) {
      (void)hipFree(p);
      mem_track(-static_cast<int64_t>(n));
    }
  }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

char* vat(void* base, size_t v64, int i) { return static_cast<char*>(base) + static_cast<size_t>(i) * v64; }

// Chiral half-vectors (Sec. V: a vector of definite chirality needs half the
// storage).  A half-vector of sector s holds the 6 complex components of
// chirality s per site, [parity][6][N/2] FP64 elements of 16 bytes: the rows
// c = 0..5 (s = +1) or 6..11 (s = -1) of the full layout [parity][12][N/2].
// The basis kernels (dots, axpys, rotations) treat a vector as a flat array
// of 16-byte elements, so a half-vector goes to them as a full vector on a
// geometry of N/2 sites (N/2 is a multiple of 8 on every valid lattice).
ovl_geom half_geom(const ovl_geom* g) {
  ovl_geom h = *g;
  h.N = g->N / 2;
  h.geo.Nh = g->geo.Nh / 2;
  return h;
}

// half <- the sector rows of the full FP64 vector f (that is, P_s f)
void to_half(void* h, const void* f, const ovl_geom* g, int sector, hipStream_t s) {
  const size_t row = static_cast<size_t>(g->geo.Nh) * 16, c0 = sector > 0 ? 0 : 6;
  OVL_HIP(hipMemcpy2DAsync(h, 6 * row, static_cast<const char*>(f) + c0 * row, 12 * row, 6 * row, 2,
                           hipMemcpyDeviceToDevice, s));
}

// the sector rows of the full FP64 vector f <- half (the other rows untouched)
void to_full(void* f, const void* h, const ovl_geom* g, int sector, hipStream_t s) {
  const size_t row = static_cast<size_t>(g->geo.Nh) * 16, c0 = sector > 0 ? 0 : 6;
  OVL_HIP(hipMemcpy2DAsync(static_cast<char*>(f) + c0 * row, 12 * row, h, 6 * row, 6 * row, 2,
                           hipMemcpyDeviceToDevice, s));
}

}  // namespace
}  // namespace ovl

using namespace ovl;

extern "C" {

int ovl_overlap_eigs(const ovl_gauge* u, double rho, const ovl_sign* sgn, const ovl_lowmodes* lm, ovl_prec prec,
                     int sector, int ell, int K, void* V, double* d, int* nout, double tol, int max_iter,
                     ovl_eig_stats* stats, ovl_stream_t st) {
  return guard([&] {
    OVL_REQUIRE(u && sgn && V && d && nout && stats, OVL_E_ARG, "null argument");
    check_prec(prec);
    {
      int recon = 0;
      gauge_links(u, prec, &recon);  // OVL_E_PRECISION before any work when prec's links are missing
    }
    OVL_REQUIRE(sector == 1 || sector == -1, OVL_E_ARG, "sector must be +1 or -1");
    OVL_REQUIRE(ell >= 1 && K >= ell + 8 && K <= 512, OVL_E_ARG, "need ell >= 1 and ell + 8 <= K <= 512");
    OVL_REQUIRE(tol > 0.0 && max_iter >= 1, OVL_E_ARG, "need tol > 0 and max_iter >= 1");
    if (lm && lm->ell == 0) lm = nullptr;
    if (lm) OVL_REQUIRE(lm->geom.N == u->geom.N, OVL_E_ARG, "low modes and gauge field have different lattices");
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = static_cast<hipStream_t>(st);
    const ovl_geom* g = &u->geom;
    const ovl_geom hg = half_geom(g);  // the Lanczos basis: chiral half-vectors
    const size_t v64 = spinor_vec_bytes(g, OVL_F64), vh = v64 / 2;
    const size_t N = static_cast<size_t>(g->N);
    *stats = ovl_eig_stats{};
    const int keep = std::max(ell + 4, std::min(K - 4, ell + (K - ell) / 2));  // thick-restart size

    DevBuf Q(vh * (K + 1)), w(vh), t(v64), xf(v64), wf(v64);
    // the sign applications at storage precision prec (FP32 arithmetic below
    // FP64): the full vector is converted in and the result back to FP64
    const size_t vp = spinor_vec_bytes(g, prec);
    DevBuf pin(prec == OVL_F64 ? 16 : vp), pout(prec == OVL_F64 ? 16 : vp);
    DevBuf sc(sizeof(double) * 4 + sizeof(int) * 2);
    double* dsc = static_cast<double*>(sc.p);
    int* dsect = reinterpret_cast<int*>(dsc + 4);
    WsBuf cb(sizeof(double2) * (K + 1), s);
    DevBuf Sdev(sizeof(double2) * static_cast<size_t>(K) * K);
    const int hsect[2] = {sector, -sector};
    OVL_HIP(hipMemcpyAsync(dsect, hsect, sizeof(hsect), hipMemcpyHostToDevice, s));
    blas_zero(xf.p, v64, s);  // the rows of chirality -s stay zero

    // norm of a vector of `bytes` bytes
    auto norm = [&](const void* x, size_t bytes) {
      blas_norm2(OVL_F64, bytes / 16, x, 1, bytes, dsc, s);
      double h[2];
      OVL_HIP(hipMemcpyAsync(h, dsc, sizeof(h), hipMemcpyDeviceToHost, s));
      OVL_HIP(hipStreamSynchronize(s));
      return std::sqrt(h[0]);
    };
    // y = a x (+ b y) on vectors of `sites` sites' worth of FP64 elements,
    // complex host scalars
    auto axpby = [&](size_t sites, const void* x, zc a, void* y, bool keep_y, zc b = zc(1.0, 0.0)) {
      const double h[4] = {a.real(), a.imag(), b.real(), b.imag()};
      OVL_HIP(hipMemcpyAsync(dsc, h, sizeof(h), hipMemcpyHostToDevice, s));
      blas_axpby(OVL_F64, x, dsc, OVL_F64, y, keep_y ? dsc + 2 : nullptr, sites, 1, s);
      OVL_HIP(hipStreamSynchronize(s));  // the host scalars are reused
    };
    // out = eps in (full FP64 vectors; the sign applied at precision prec), counted
    auto eps = [&](void* out, const void* in) {
      if (prec == OVL_F64) {
        overlap_apply(out, in, u, rho, 0.0, sgn, lm, 0, OVL_F64, 1, s);
      } else {
        blas_convert(OVL_F64, in, prec, pin.p, N, 1, s);
        overlap_apply(pout.p, pin.p, u, rho, 0.0, sgn, lm, 0, prec, 1, s);
        blas_convert(prec, pout.p, OVL_F64, out, N, 1, s);
      }
      stats->hw_applies += 2 * (static_cast<int64_t>(sgn->c.size()) - 1) + 1;
    };
    // below this partner norm a pair is taken for a real mode: FP64 rounding,
    // or the noise of a lower-precision sign
    const double real_mode_sn = prec == OVL_F64 ? 1e-9 : 1e-5;
    // out = K_s in = s P_s eps in, on half-vectors
    auto apply_K = [&](void* out, const void* in) {
      to_full(xf.p, in, g, sector, s);
      eps(t.p, xf.p);
      to_half(out, t.p, g, sector, s);
      if (sector < 0) axpby(N / 2, out, zc(-1.0, 0.0), out, false);
    };
    auto upload_S = [&](const std::vector<zc>& S, int rows, int cols) {
      std::vector<double2> h(static_cast<size_t>(rows) * cols);
      for (size_t i = 0; i < h.size(); ++i) h[i] = make_double2(S[i].real(), S[i].imag());
      OVL_HIP(hipMemcpyAsync(Sdev.p, h.data(), h.size() * sizeof(double2), hipMemcpyHostToDevice, s));
      OVL_HIP(hipStreamSynchronize(s));
    };

    // q_0: the sector part of the caller's start vector
    to_half(Q.p, V, g, sector, s);
    {
      const double n0 = norm(Q.p, vh);
      OVL_REQUIRE(n0 > 0.0 && std::isfinite(n0), OVL_E_ARG, "start vector has no component in the sector");
      axpby(N / 2, Q.p, zc(1.0 / n0, 0.0), Q.p, false);
    }
    std::vector<zc> T(static_cast<size_t>(K + 1) * (K + 1), zc(0.0, 0.0));
    auto Tat = [&](int i, int j) -> zc& { return T[i + static_cast<size_t>(K + 1) * j]; };
    std::vector<double2> hc(K + 1), hc2(K + 1);
    std::vector<double> th;
    std::vector<zc> S;
    int cur = 0;
    double worst = INFINITY;
    for (int cycle = 0;; ++cycle) {
      for (int j = cur; j < K; ++j) {
        apply_K(w.p, vat(Q.p, vh, j));
        for (int i = 0; i <= j; ++i) hc2[i] = make_double2(0.0, 0.0);
        for (int pass = 0; pass < 2; ++pass) {  // w -= Q (Q^dag w), twice
          block_dot(&hg, Q.p, j + 1, w.p, OVL_F64, 1, static_cast<double2*>(cb.p), s);
          OVL_HIP(hipMemcpyAsync(hc.data(), cb.p, sizeof(double2) * (j + 1), hipMemcpyDeviceToHost, s));
          OVL_HIP(hipStreamSynchronize(s));
          for (int i = 0; i <= j; ++i) {
            hc2[i] = make_double2(hc2[i].x + hc[i].x, hc2[i].y + hc[i].y);
            hc[i] = make_double2(-hc[i].x, -hc[i].y);
          }
          OVL_HIP(hipMemcpyAsync(cb.p, hc.data(), sizeof(double2) * (j + 1), hipMemcpyHostToDevice, s));
          block_axpy(&hg, Q.p, j + 1, static_cast<const double2*>(cb.p), w.p, OVL_F64, 1, true, s);
          OVL_HIP(hipStreamSynchronize(s));
        }
        for (int i = 0; i <= j; ++i) Tat(i, j) = zc(hc2[i].x, hc2[i].y);
        const double beta = norm(w.p, vh);
        OVL_REQUIRE(std::isfinite(beta), OVL_E_NAN, "overlap eigensolver: NaN in the Lanczos recurrence");
        if (beta == 0.0) throw Error(OVL_E_BREAKDOWN, "overlap eigensolver: invariant subspace found before K steps");
        Tat(j + 1, j) = beta;
        axpby(N / 2, w.p, zc(1.0 / beta, 0.0), vat(Q.p, vh, j + 1), false);
      }
      // Ritz pairs, lowest first; residual ||K y - theta y|| = beta_K |s_{K-1}|
      std::vector<zc> Tk(static_cast<size_t>(K) * K);
      for (int j = 0; j < K; ++j)
        for (int i = 0; i < K; ++i) Tk[i + static_cast<size_t>(K) * j] = 0.5 * (Tat(i, j) + std::conj(Tat(j, i)));
      host_heev(K, Tk, th, S);
      const double betaK = Tat(K, K - 1).real();
      worst = 0.0;
      for (int i = 0; i < ell; ++i) worst = std::max(worst, betaK * std::abs(S[(K - 1) + static_cast<size_t>(K) * i]));
      stats->iterations = cycle + 1;
      if (log_on())
        fprintf(stderr, "[ovl overlap eigs] cycle %d (basis %d): max Ritz residual %.3e, k_%d = %.6f\n", cycle, K, worst,
                ell, th[ell - 1]);
      if (worst <= tol || cycle + 1 >= max_iter) break;
      // thick restart: the `keep` lowest Ritz vectors and the residual direction
      upload_S(S, K, K);
      block_rotate_inplace(&hg, Q.p, K, static_cast<const double2*>(Sdev.p), keep, s);
      OVL_HIP(hipMemcpyAsync(vat(Q.p, vh, keep), vat(Q.p, vh, K), vh, hipMemcpyDeviceToDevice, s));
      std::fill(T.begin(), T.end(), zc(0.0, 0.0));
      for (int i = 0; i < keep; ++i) {
        Tat(i, i) = th[i];
        const zc c = betaK * S[(K - 1) + static_cast<size_t>(K) * i];
        Tat(keep, i) = c;
        Tat(i, keep) = std::conj(c);
      }
      cur = keep;
    }
    // the ell lowest Ritz vectors, then the pairs of D from each of them;
    // vector i of the sector sits in Q[i] after the rotation
    upload_S(S, K, K);
    block_rotate_inplace(&hg, Q.p, K, static_cast<const double2*>(Sdev.p), ell, s);
    int n = 0;
    double max_res = 0.0;
    const double r2 = 1.0 / std::sqrt(2.0);
    for (int i = 0; i < ell; ++i) {
      to_full(xf.p, vat(Q.p, vh, i), g, sector, s);  // v as a full vector
      eps(t.p, xf.p);
      // wf = P_{-s} eps v (the partner direction), t = P_s eps v
      OVL_HIP(hipMemcpyAsync(wf.p, t.p, v64, hipMemcpyDeviceToDevice, s));
      blas_chiral(OVL_F64, v64, wf.p, 1, dsect + 1, s);
      blas_chiral(OVL_F64, v64, t.p, 1, dsect, s);
      // explicit residual ||s P_s eps v - k v||
      axpby(N, xf.p, zc(-sector * th[i], 0.0), t.p, true);
      max_res = std::max(max_res, norm(t.p, v64));
      const double sn = norm(wf.p, v64);
      const double k = std::min(1.0, std::max(-1.0, th[i]));
      if (sn <= real_mode_sn) {  // real mode of chirality `sector`
        OVL_HIP(hipMemcpyAsync(vat(V, v64, n), xf.p, v64, hipMemcpyDeviceToDevice, s));
        d[2 * n] = 1.0 + k;
        d[2 * n + 1] = 0.0;
        ++n;
        continue;
      }
      // xi = (v + sg i u)/sqrt(2), d = 1 + k + sg i s sn; negative imaginary part first
      for (int half = 0; half < 2; ++half) {
        const int sg = (half == 0) ? -sector : sector;
        void* xo = vat(V, v64, n);
        axpby(N, xf.p, zc(r2, 0.0), xo, false);
        axpby(N, wf.p, zc(0.0, sg * r2 / sn), xo, true);
        d[2 * n] = 1.0 + k;
        d[2 * n + 1] = sg * sector * sn;
        ++n;
      }
    }
    OVL_HIP(hipStreamSynchronize(s));
    *nout = n;
    stats->max_residual = max_res;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (log_on())
      fprintf(stderr, "[ovl overlap eigs] %d eigenpairs of D from %d sector vectors, max residual %.3e, %.1f s\n", n,
              ell, max_res, stats->seconds);
    return max_res <= tol ? OVL_OK : OVL_W_NOT_CONVERGED;
  });
}

int ovl_deflation_create(const ovl_geom* g, int n, const void* Xi, const double* d, ovl_deflation** out) {
  return guard([&] {
    OVL_REQUIRE(g && Xi && d && out, OVL_E_ARG, "null argument");
    OVL_REQUIRE(n >= 1 && n <= 4096, OVL_E_ARG, "need 1 <= n <= 4096 eigenpairs");
    ovl_deflation* df = new ovl_deflation;
    df->geom = *g;
    df->n = n;
    df->Xi = Xi;
    df->d.resize(n);
    for (int i = 0; i < n; ++i) {
      df->d[i] = zc(d[2 * i], d[2 * i + 1]);
      if (!std::isfinite(d[2 * i]) || !std::isfinite(d[2 * i + 1])) {
        delete df;
        throw Error(OVL_E_NAN, "non-finite eigenvalue");
      }
    }
    *out = df;
    return OVL_OK;
  });
}

int ovl_deflation_destroy(ovl_deflation* df) {
  delete df;
  return OVL_OK;
}

int ovl_deflation_prepare(ovl_deflation* df, const ovl_gauge* u, double rho, const ovl_sign* sgn,
                          const ovl_lowmodes* lm, void* Z, ovl_stream_t st) {
  return guard([&] {
    OVL_REQUIRE(df && u && sgn && Z, OVL_E_ARG, "null argument");
    OVL_REQUIRE(df->geom.N == u->geom.N, OVL_E_ARG, "deflation and gauge field have different lattices");
    OVL_REQUIRE(rho > 0.0 && std::isfinite(rho), OVL_E_ARG, "need rho > 0");
    OVL_REQUIRE(Z != df->Xi, OVL_E_ALIAS, "Z must not be the eigenvector buffer");
    if (lm && lm->ell == 0) lm = nullptr;
    if (lm) OVL_REQUIRE(lm->geom.N == u->geom.N, OVL_E_ARG, "low modes and gauge field have different lattices");
    hipStream_t s = static_cast<hipStream_t>(st);
    const ovl_geom* g = &df->geom;
    const int n = df->n;
    const size_t v64 = spinor_vec_bytes(g, OVL_F64);
    auto at = [&](const void* base, int i) { return static_cast<const char*>(base) + static_cast<size_t>(i) * v64; };
    // Z = D(0) Xi = rho D Xi, in batches of up to 12 vectors
    for (int i0 = 0; i0 < n; i0 += OVL_MAX_RHS) {
      const int nb = std::min(OVL_MAX_RHS, n - i0);
      overlap_apply(static_cast<char*>(Z) + static_cast<size_t>(i0) * v64, at(df->Xi, i0), u, rho, 0.0, sgn, lm,
                    1 /* D(m) */, OVL_F64, nb, s);
    }
    // Gram matrices, column by column in batches of up to 12
    WsBuf cb(sizeof(double2) * static_cast<size_t>(n) * OVL_MAX_RHS, s);
    std::vector<double2> h(static_cast<size_t>(n) * OVL_MAX_RHS);
    std::vector<zc> ZZ(static_cast<size_t>(n) * n), ZX(ZZ.size()), XX(ZZ.size());
    auto gram = [&](const void* A, const void* B, std::vector<zc>& out) {  // out[i + n j] = A_i^dag B_j
      for (int j0 = 0; j0 < n; j0 += OVL_MAX_RHS) {
        const int nb = std::min(OVL_MAX_RHS, n - j0);
        block_dot(g, A, n, at(B, j0), OVL_F64, nb, static_cast<double2*>(cb.p), s);
        OVL_HIP(hipMemcpyAsync(h.data(), cb.p, sizeof(double2) * static_cast<size_t>(n) * nb, hipMemcpyDeviceToHost, s));
        OVL_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < n; ++i)
          for (int r = 0; r < nb; ++r) {
            const double2 c = h[static_cast<size_t>(i) * nb + r];
            OVL_REQUIRE(std::isfinite(c.x) && std::isfinite(c.y), OVL_E_NAN, "non-finite Gram matrix entry");
            out[i + static_cast<size_t>(n) * (j0 + r)] = zc(c.x, c.y);
          }
      }
    };
    gram(Z, Z, ZZ);
    gram(Z, df->Xi, ZX);
    gram(df->Xi, df->Xi, XX);
    df->Z = Z;
    df->rho = rho;
    df->ZZ.swap(ZZ);
    df->ZX.swap(ZX);
    df->XX.swap(XX);
    return OVL_OK;
  });
}

}  // extern "C"

namespace ovl {

namespace {

// Solves the n x n complex system A Y = B for R right-hand sides in place
// (Gaussian elimination with partial pivoting; A column-major, B[i*R + r]).
void host_solve(std::vector<zc>& A, std::vector<zc>& B, int n, int R) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int i = c + 1; i < n; ++i)
      if (std::abs(A[i + static_cast<size_t>(n) * c]) > std::abs(A[piv + static_cast<size_t>(n) * c])) piv = i;
    OVL_REQUIRE(std::abs(A[piv + static_cast<size_t>(n) * c]) > 0.0, OVL_E_BREAKDOWN,
                "deflation: singular projected system (linearly dependent eigenvectors)");
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c + static_cast<size_t>(n) * k], A[piv + static_cast<size_t>(n) * k]);
      for (int r = 0; r < R; ++r) std::swap(B[static_cast<size_t>(c) * R + r], B[static_cast<size_t>(piv) * R + r]);
    }
    const zc dgn = A[c + static_cast<size_t>(n) * c];
    for (int i = c + 1; i < n; ++i) {
      const zc f = A[i + static_cast<size_t>(n) * c] / dgn;
      if (f == zc(0.0, 0.0)) continue;
      for (int k = c; k < n; ++k) A[i + static_cast<size_t>(n) * k] -= f * A[c + static_cast<size_t>(n) * k];
      for (int r = 0; r < R; ++r) B[static_cast<size_t>(i) * R + r] -= f * B[static_cast<size_t>(c) * R + r];
    }
  }
  for (int i = n - 1; i >= 0; --i)
    for (int r = 0; r < R; ++r) {
      zc v = B[static_cast<size_t>(i) * R + r];
      for (int k = i + 1; k < n; ++k) v -= A[i + static_cast<size_t>(n) * k] * B[static_cast<size_t>(k) * R + r];
      B[static_cast<size_t>(i) * R + r] = v / A[i + static_cast<size_t>(n) * i];
    }
}

}  // namespace

// The low part of eq. 9 for a batch of FP64 residuals r (R vectors):
// x += sum_i xi_i (xi_i^dag r) / (rho d_i + m (1 - d_i / 2)),
// r -= sum_i xi_i (xi_i^dag r).
// After ovl_deflation_prepare, the minimal-residual form instead: with
// W = D(m) Xi = a Z + m Xi (a = 1 - m / (2 rho), Z = D(0) Xi), the y that
// minimises ||r - W y|| solves (W^dag W) y = W^dag r; then x += Xi y and
// r -= W y, which is r's exact update.  For exact eigenpairs (orthonormal,
// W = Xi diag(d(m))) both forms give the same y.
void deflate(const ovl_deflation* df, double rho, double m, void* x, void* r, int R, hipStream_t s) {
  const ovl_geom* g = &df->geom;
  const int n = df->n;
  WsBuf cbuf(sizeof(double2) * static_cast<size_t>(n) * R, s);
  double2* C = static_cast<double2*>(cbuf.p);
  if (df->Z) {
    const double a = 1.0 - m / (2.0 * rho);
    WsBuf cbuf2(sizeof(double2) * static_cast<size_t>(n) * R, s);
    block_dot(g, df->Xi, n, r, OVL_F64, R, C, s);
    block_dot(g, df->Z, n, r, OVL_F64, R, static_cast<double2*>(cbuf2.p), s);
    std::vector<double2> h1(static_cast<size_t>(n) * R), h2(h1.size());
    OVL_HIP(hipMemcpyAsync(h1.data(), C, sizeof(double2) * h1.size(), hipMemcpyDeviceToHost, s));
    OVL_HIP(hipMemcpyAsync(h2.data(), cbuf2.p, sizeof(double2) * h2.size(), hipMemcpyDeviceToHost, s));
    OVL_HIP(hipStreamSynchronize(s));
    std::vector<zc> G(static_cast<size_t>(n) * n), Y(h1.size());
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const size_t ij = i + static_cast<size_t>(n) * j, ji = j + static_cast<size_t>(n) * i;
        G[ij] = a * a * df->ZZ[ij] + a * m * (df->ZX[ij] + std::conj(df->ZX[ji])) + m * m * df->XX[ij];
      }
    for (size_t k = 0; k < Y.size(); ++k) Y[k] = a * zc(h2[k].x, h2[k].y) + m * zc(h1[k].x, h1[k].y);
    host_solve(G, Y, n, R);
    std::vector<double2> kx(Y.size()), kz(Y.size()), kr(Y.size());
    for (size_t k = 0; k < Y.size(); ++k) {
      kx[k] = make_double2(Y[k].real(), Y[k].imag());
      kz[k] = make_double2(-a * Y[k].real(), -a * Y[k].imag());
      kr[k] = make_double2(-m * Y[k].real(), -m * Y[k].imag());
    }
    WsBuf dx(sizeof(double2) * kx.size(), s), dz(sizeof(double2) * kz.size(), s), dr(sizeof(double2) * kr.size(), s);
    OVL_HIP(hipMemcpyAsync(dx.p, kx.data(), sizeof(double2) * kx.size(), hipMemcpyHostToDevice, s));
    OVL_HIP(hipMemcpyAsync(dz.p, kz.data(), sizeof(double2) * kz.size(), hipMemcpyHostToDevice, s));
    OVL_HIP(hipMemcpyAsync(dr.p, kr.data(), sizeof(double2) * kr.size(), hipMemcpyHostToDevice, s));
    block_axpy(g, df->Xi, n, static_cast<const double2*>(dx.p), x, OVL_F64, R, true, s);
    block_axpy(g, df->Z, n, static_cast<const double2*>(dz.p), r, OVL_F64, R, true, s);
    block_axpy(g, df->Xi, n, static_cast<const double2*>(dr.p), r, OVL_F64, R, true, s);
    OVL_HIP(hipStreamSynchronize(s));  // the host coefficient arrays end with this scope
    return;
  }
  block_dot(g, df->Xi, n, r, OVL_F64, R, C, s);
  std::vector<double2> h(static_cast<size_t>(n) * R), hx(h.size());
  OVL_HIP(hipMemcpyAsync(h.data(), C, sizeof(double2) * h.size(), hipMemcpyDeviceToHost, s));
  OVL_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < n; ++i) {
    const zc lam = rho * df->d[i] + m * (1.0 - 0.5 * df->d[i]);
    for (int r2 = 0; r2 < R; ++r2) {
      const size_t k = static_cast<size_t>(i) * R + r2;
      const zc c(h[k].x, h[k].y);
      const zc q = c / lam;
      hx[k] = make_double2(q.real(), q.imag());
      h[k] = make_double2(-c.real(), -c.imag());
    }
  }
  WsBuf kx(sizeof(double2) * hx.size(), s), kr(sizeof(double2) * h.size(), s);
  OVL_HIP(hipMemcpyAsync(kx.p, hx.data(), sizeof(double2) * hx.size(), hipMemcpyHostToDevice, s));
  OVL_HIP(hipMemcpyAsync(kr.p, h.data(), sizeof(double2) * h.size(), hipMemcpyHostToDevice, s));
  block_axpy(g, df->Xi, n, static_cast<const double2*>(kx.p), x, OVL_F64, R, true, s);
  block_axpy(g, df->Xi, n, static_cast<const double2*>(kr.p), r, OVL_F64, R, true, s);
  OVL_HIP(hipStreamSynchronize(s));  // the host coefficient arrays end with this scope
}

}  // namespace ovl
