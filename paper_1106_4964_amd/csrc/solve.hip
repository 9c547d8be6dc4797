// CG for quark propagators (arXiv:1106.4964 Sec. II, Sec. V).
//
// Solves D(m) x = b for a batch of right-hand sides by CG on
// A = D(m) D(m)^dag with x = D(m)^dag y (Craig's method), so the recursively
// updated residual is b - D(m) x.  An outer loop recomputes the true
// residual in FP64 and restarts the inner solve on it (defect correction)
// until every rhs has ||b - D(m) x|| <= tol ||b||.  The inner solve runs at
// the storage precision the caller asks for (FP64 gives plain FP64 CG); its
// correction is accumulated in FP64.
//
// Every Krylov scalar lives on the device: reductions write FP64 results to
// device memory, tiny kernels turn them into alpha/beta and per-rhs
// activity masks, and the vector kernels read them from there.  Nothing in
// an inner iteration needs the host, so a chunk of iterations can be
// captured once in a HIP graph and replayed; the host only reads the masks
// between replays.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "ops.h"

namespace ovl {
namespace {

// Scalars of one inner solve, all device-resident, one slot per rhs.
struct Scalars {
  double rr[OVL_MAX_RHS];
  double rrn[OVL_MAX_RHS];
  double pp[OVL_MAX_RHS];
  double target[OVL_MAX_RHS];
  double alpha[2 * OVL_MAX_RHS];   // complex (a, 0)
  double malpha[2 * OVL_MAX_RHS];  // complex (-a, 0)
  double beta[2 * OVL_MAX_RHS];
  double tcoef[2 * OVL_MAX_RHS];   // weight of the new gradient in p (0 = p frozen)
  double one[2 * OVL_MAX_RHS];
  double mone[2 * OVL_MAX_RHS];
  double scale[2 * OVL_MAX_RHS];   // rhs scale factors of the inner system
  double iscale[2 * OVL_MAX_RHS];
  double dot_tmp[2 * OVL_MAX_RHS];
  int active[OVL_MAX_RHS];
  int bad[OVL_MAX_RHS];  // 1 breakdown (p^dag p <= 0), 2 NaN/Inf
  int sector[OVL_MAX_RHS];  // chiral inner solves: +1 or -1 per rhs
};

// dot results arrive as (re, im) pairs; keep the real parts.
__global__ void take_real_kernel(int R, const double* d, double* out) {
  const int r = threadIdx.x;
  if (r < R) out[r] = d[2 * r];
}

__global__ void alpha_kernel(int R, Scalars* S) {
  const int r = threadIdx.x;
  if (r >= R) return;
  double a = 0.0;
  if (S->active[r]) {
    const double pp = S->pp[r], rr = S->rr[r];
    if (!(pp == pp) || !(rr == rr) || isinf(pp) || isinf(rr)) {
      S->bad[r] = 2;
      S->active[r] = 0;
    } else if (pp <= 0.0) {
      S->bad[r] = 1;
      S->active[r] = 0;
    } else {
      a = rr / pp;
    }
  }
  S->alpha[2 * r] = a;
  S->alpha[2 * r + 1] = 0.0;
  S->malpha[2 * r] = -a;
  S->malpha[2 * r + 1] = 0.0;
}

// p = tcoef * g + beta * p with g the new gradient.  A rhs that reaches its
// target takes this step's direction update; from then on p is frozen
// (tcoef 0, beta 1) while alpha = 0 leaves its iterate alone.
__global__ void beta_kernel(int R, Scalars* S) {
  const int r = threadIdx.x;
  if (r >= R) return;
  double b = 1.0, tc = 0.0;
  if (S->active[r]) {
    const double rrn = S->rrn[r];
    if (!(rrn == rrn) || isinf(rrn)) {
      S->bad[r] = 2;
      S->active[r] = 0;
      b = 0.0;
    } else {
      b = rrn / S->rr[r];
      tc = 1.0;
      S->rr[r] = rrn;
      if (rrn <= S->target[r]) S->active[r] = 0;
    }
  }
  S->beta[2 * r] = b;
  S->beta[2 * r + 1] = 0.0;
  S->tcoef[2 * r] = tc;
  S->tcoef[2 * r + 1] = 0.0;
}

struct Solver {
  const ovl_gauge* u;
  double rho, m;
  const ovl_sign* sg;      // outer (FP64 true residual)
  const ovl_sign* sg_in;   // inner operator
  const ovl_lowmodes* lm;
  int R, P;
  hipStream_t s;
  size_t v64, vP, nsites;
  ovl_solve_stats* st;
  int64_t per_sign_dw, per_sign_dw_in;

  // inner = true: the inner operator (relaxed sign), else the FP64 one
  void dm(void* out, const void* in, int prec, int dagger, bool inner) {
    overlap_apply(out, in, u, rho, m, inner ? sg_in : sg, lm, dagger ? 2 : 1, prec, R, s);
    st->sign_applies += R;
    st->dslash_applies += R * (inner ? per_sign_dw_in : per_sign_dw);
  }
  // chiral sector operator: out = P_s [c0 in + c1 gamma5 sign(H_w) in] for
  // in = P_s in, which is D(m) D(m)^dag in when sign^2 = 1
  void achiral(void* out, const void* in, int prec, Scalars* S) {
    const double c0 = 2.0 * rho * rho + 0.5 * m * m, c1 = 2.0 * (rho * rho - 0.25 * m * m);
    overlap_combine(out, in, u, rho, c0, c1, sg_in, lm, prec, R, s);
    blas_chiral(prec, vP, out, R, S->sector, s);
    st->sign_applies += R;
    st->dslash_applies += R * per_sign_dw_in;
  }
  // real part of p^dag q per rhs
  void rdot(const void* x, const void* y, int prec, double* dev_out, Scalars* S) {
    blas_dot(prec, (prec == OVL_F64 ? v64 : vP) / 16, x, y, R, prec == OVL_F64 ? v64 : vP, S->dot_tmp, s);
    hipLaunchKernelGGL(take_real_kernel, dim3(1), dim3(64), 0, s, R, S->dot_tmp, dev_out);
  }
  void norm2(const void* x, int prec, double* dev_out, Scalars* S) {
    blas_norm2(prec, (prec == OVL_F64 ? v64 : vP) / 16, x, R, prec == OVL_F64 ? v64 : vP, S->dot_tmp, s);
    hipLaunchKernelGGL(take_real_kernel, dim3(1), dim3(64), 0, s, R, S->dot_tmp, dev_out);
  }
};

}  // namespace

int cg_solve(void* x, const void* b, int R, const ovl_gauge* u, double rho, double m, const ovl_sign* sg,
             const ovl_lowmodes* lm, double tol, int maxiter, const ovl_solve_opts* o, ovl_solve_stats* st,
             hipStream_t us) {
  const auto t_start = std::chrono::steady_clock::now();
  ovl_solve_opts def{};
  def.inner_prec = OVL_F64;
  def.inner_tol = 0.0;
  def.graph_chunk = 0;
  def.check_every = 1;
  def.max_restarts = 50;
  const ovl_solve_opts& opt = o ? *o : def;
  const int P = opt.inner_prec;
  check_prec(P);
  const int check_every = std::max(1, opt.check_every);
  // chiral inner solves; switched off for the rest of the solve when a
  // chiral cycle breaks down or fails to halve the true residual (the
  // sector operator is only positive to within the sign error times
  // 2 rho^2, which must stay below m^2)
  bool chiral = opt.chiral != 0;
  OVL_REQUIRE(!chiral || !(opt.harvest_x && opt.harvest_b && opt.harvest_cap > 0), OVL_E_ARG,
              "chiral solves do not harvest training pairs");
  OVL_REQUIRE(!chiral || !opt.deflation, OVL_E_ARG, "chiral solves do not take a deflation");
  if (opt.deflation) {
    OVL_REQUIRE(opt.deflation->geom.N == u->geom.N, OVL_E_ARG, "deflation and gauge field have different lattices");
    OVL_REQUIRE(!opt.deflation->Z || opt.deflation->rho == rho, OVL_E_ARG,
                "the deflation was prepared with another rho");
  }

  Solver S{};
  S.u = u;
  S.rho = rho;
  S.m = m;
  S.sg = sg;
  S.lm = lm;
  S.R = R;
  S.P = P;
  S.st = st;
  S.nsites = static_cast<size_t>(u->geom.N);
  S.v64 = spinor_vec_bytes(&u->geom, OVL_F64);
  S.vP = spinor_vec_bytes(&u->geom, P);
  S.per_sign_dw = 2 * (static_cast<int64_t>(sg->c.size()) - 1) + 1;
  S.sg_in = (o && o->inner_sign) ? o->inner_sign : sg;
  OVL_REQUIRE(S.sg_in->lam_max == sg->lam_max, OVL_E_ARG, "inner_sign must share lam_max with sign");
  S.per_sign_dw_in = 2 * (static_cast<int64_t>(S.sg_in->c.size()) - 1) + 1;
  int recon = 0;
  (void)gauge_links(u, P, &recon);  // the inner precision must have links
  // adaptive precision: the inner sign and the coarser ones the solve may
  // switch to as the inner residual drops
  std::vector<const ovl_sign*> ladder{S.sg_in};
  if (opt.relax_signs && opt.n_relax > 0) {
    OVL_REQUIRE(!chiral, OVL_E_ARG, "relaxed inner signs do not combine with chiral solves");
    OVL_REQUIRE(opt.n_relax <= 8, OVL_E_ARG, "at most 8 relax signs");
    for (int k = 0; k < opt.n_relax; ++k) {
      const ovl_sign* rs = opt.relax_signs[k];
      OVL_REQUIRE(rs && rs->lam_max == sg->lam_max, OVL_E_ARG, "relax signs must share lam_max with sign");
      OVL_REQUIRE(rs->delta > ladder.back()->delta, OVL_E_ARG, "relax signs must have increasing delta");
      ladder.push_back(rs);
    }
  }
  int level = 0;
  auto set_level = [&](int lv) {
    level = lv;
    S.sg_in = ladder[lv];
    S.per_sign_dw_in = 2 * (static_cast<int64_t>(S.sg_in->c.size()) - 1) + 1;
  };

  // private stream (graph capture needs one), ordered after the caller's work
  hipStream_t s;
  OVL_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  S.s = s;
  hipEvent_t ev;
  OVL_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  OVL_HIP(hipEventRecord(ev, us));
  OVL_HIP(hipStreamWaitEvent(s, ev, 0));
  // s now runs after everything queued on the caller's stream, so the free
  // workspace kept for that stream can serve this solve
  ws_retire_stream(us, s);

  // one captured chunk per inner sign (the sign's coefficients are kernel
  // arguments); a chunk captured for the chiral operator is recaptured when
  // the solve leaves chiral mode
  std::vector<hipGraphExec_t> gexecs(ladder.size(), nullptr);
  std::vector<hipGraph_t> graphs(ladder.size(), nullptr);
  std::vector<char> graph_chiral(ladder.size(), 0);
  auto drop_graphs = [&]() {
    for (size_t k = 0; k < ladder.size(); ++k) {
      if (gexecs[k]) (void)hipGraphExecDestroy(gexecs[k]);
      if (graphs[k]) (void)hipGraphDestroy(graphs[k]);
      gexecs[k] = nullptr;
      graphs[k] = nullptr;
    }
  };
  int rc = OVL_OK;
  try {
    WsBuf r64(S.v64 * R, s), tmp64(S.v64 * R, s), e64(S.v64 * R, s);
    WsBuf rin(S.vP * R, s), p(S.vP * R, s), q(S.vP * R, s), t(S.vP * R, s);
    WsBuf sbuf(sizeof(Scalars), s);
    Scalars* dS = static_cast<Scalars*>(sbuf.p);
    Scalars hS{};
    bool capturing = false;
    for (int r = 0; r < R; ++r) {
      hS.one[2 * r] = 1.0;
      hS.mone[2 * r] = -1.0;
    }
    OVL_HIP(hipMemcpyAsync(dS, &hS, sizeof(Scalars), hipMemcpyHostToDevice, s));
    OVL_HIP(hipStreamSynchronize(s));

    // ||b||^2
    std::vector<double> bn2(R), rn2(R);
    S.norm2(b, OVL_F64, dS->rrn, dS);
    OVL_HIP(hipMemcpyAsync(&hS.rrn, dS->rrn, sizeof(double) * R, hipMemcpyDeviceToHost, s));
    OVL_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < R; ++r) {
      bn2[r] = hS.rrn[r];
      OVL_REQUIRE(std::isfinite(bn2[r]), OVL_E_NAN, "right-hand side contains NaN or Inf");
    }

    // exact pairs (x = p_r, b = D(m) p_r) for training, outside graphs only
    const bool harvest = opt.harvest_x && opt.harvest_b && opt.harvest_cap > 0;
    const size_t v32 = spinor_vec_bytes(&u->geom, OVL_F32);
    auto harvest_pairs = [&]() {
      for (int r = 0; r < R && st->harvested < opt.harvest_cap; ++r) {
        if (!hS.active[r]) continue;
        blas_convert(P, static_cast<char*>(p.p) + r * S.vP, OVL_F32,
                     static_cast<char*>(opt.harvest_x) + st->harvested * v32, S.nsites, 1, s);
        blas_convert(P, static_cast<char*>(q.p) + r * S.vP, OVL_F32,
                     static_cast<char*>(opt.harvest_b) + st->harvested * v32, S.nsites, 1, s);
        ++st->harvested;
      }
    };

    const int hstride = std::max(1, opt.harvest_stride);
    int hv_it = 0;
    // inner-iteration body; records nothing but kernel launches
    auto body = [&]() {
      S.norm2(p.p, P, dS->pp, dS);
      hipLaunchKernelGGL(alpha_kernel, dim3(1), dim3(64), 0, s, R, dS);
      blas_axpby(P, p.p, dS->alpha, OVL_F64, e64.p, dS->one, S.nsites, R, s);
      S.dm(q.p, p.p, P, 0, true);
      if (harvest && !capturing && hv_it++ % hstride == 0) harvest_pairs();
      blas_axpby(P, q.p, dS->malpha, P, rin.p, dS->one, S.nsites, R, s);
      S.norm2(rin.p, P, dS->rrn, dS);
      hipLaunchKernelGGL(beta_kernel, dim3(1), dim3(64), 0, s, R, dS);
      S.dm(t.p, rin.p, P, 1, true);
      blas_axpby(P, t.p, dS->tcoef, P, p.p, dS->beta, S.nsites, R, s);
    };

    // chiral inner iteration: CG on A = P_s D D^dag P_s for y (e64 holds y)
    auto body_chiral = [&]() {
      S.achiral(q.p, p.p, P, dS);
      S.rdot(p.p, q.p, P, dS->pp, dS);
      hipLaunchKernelGGL(alpha_kernel, dim3(1), dim3(64), 0, s, R, dS);
      blas_axpby(P, p.p, dS->alpha, OVL_F64, e64.p, dS->one, S.nsites, R, s);
      blas_axpby(P, q.p, dS->malpha, P, rin.p, dS->one, S.nsites, R, s);
      S.norm2(rin.p, P, dS->rrn, dS);
      hipLaunchKernelGGL(beta_kernel, dim3(1), dim3(64), 0, s, R, dS);
      blas_axpby(P, rin.p, dS->tcoef, P, p.p, dS->beta, S.nsites, R, s);
    };

    const double rms_target = P == OVL_F64 ? 1.0 : std::sqrt(12.0 * S.nsites) / 8.0;
    // eq. 9 deflation, dropped for the rest of the solve when a cycle ends
    // with a larger true residual than it started with: the eigenpairs are
    // then too inaccurate (1/d(m) amplifies their error instead of removing
    // the low modes), and x goes back to its value before that cycle
    const ovl_deflation* defl = opt.deflation;
    WsBuf xsave(defl ? S.v64 * R : 16, s);
    double defl_prev = INFINITY;  // worst true residual at the last cycle start
    int its = 0;
    bool chiral_failed = false;
    double prev_worst_chiral = 0.0;
    // adaptive precision: error constant of a correction per unit sign error
    // (conservative start: the first cycle runs with the finest inner sign)
    const double k_sign_min = 1.0;
    double k_sign = INFINITY, prev_worst = 0.0, cycle_delta = ladder[0]->delta;
    st->restarts = 0;
    for (;;) {
      // true residual r = b - D(m) x in FP64
      S.dm(tmp64.p, x, OVL_F64, 0, false);
      blas_axpby(OVL_F64, b, dS->one, OVL_F64, r64.p, nullptr, S.nsites, R, s);
      blas_axpby(OVL_F64, tmp64.p, dS->mone, OVL_F64, r64.p, dS->one, S.nsites, R, s);
      S.norm2(r64.p, OVL_F64, dS->rrn, dS);
      OVL_HIP(hipMemcpyAsync(rn2.data(), dS->rrn, sizeof(double) * R, hipMemcpyDeviceToHost, s));
      OVL_HIP(hipStreamSynchronize(s));
      bool done = true;
      double worst = 0.0;
      for (int r = 0; r < R; ++r) {
        const double res = bn2[r] > 0 ? std::sqrt(rn2[r] / bn2[r]) : 0.0;
        OVL_REQUIRE(std::isfinite(res), OVL_E_NAN, "true residual is NaN or Inf");
        st->true_residual[r] = res;
        worst = std::max(worst, res);
        if (res > tol) done = false;
      }
      if (log_on())
        fprintf(stderr, "[ovl cg] cycle %d: %d iterations, max FP64 true residual %.3e\n", st->restarts, its, worst);
      if (ladder.size() > 1 && prev_worst > 0.0) {
        // adaptive precision: a cycle run with sign error delta reduced the
        // residual by f; f / delta bounds the error constant of the
        // correction (from above when the cycle was limited by inner_tol)
        const double f = worst / prev_worst;
        k_sign = f < 0.5 ? std::max(k_sign_min, f / cycle_delta) : INFINITY;
      }
      prev_worst = worst;
      if (done) break;
      if (defl) {
        if (worst > defl_prev) {
          defl = nullptr;
          st->deflation_dropped = 1;
          if (log_on())
            fprintf(stderr, "[ovl cg] deflated cycle raised the residual (%.3e -> %.3e): deflation dropped\n",
                    defl_prev, worst);
          OVL_HIP(hipMemcpyAsync(x, xsave.p, S.v64 * R, hipMemcpyDeviceToDevice, s));
          prev_worst = 0.0;
          continue;  // the true residual of the restored x
        }
        OVL_HIP(hipMemcpyAsync(xsave.p, x, S.v64 * R, hipMemcpyDeviceToDevice, s));
        defl_prev = worst;
      }
      if (defl) {
        // eq. 9: the low part of the correction at once; the inner solve is
        // left with the residual minus its components along the eigenvectors
        deflate(defl, rho, m, x, r64.p, R, s);
        S.norm2(r64.p, OVL_F64, dS->rrn, dS);
        OVL_HIP(hipMemcpyAsync(rn2.data(), dS->rrn, sizeof(double) * R, hipMemcpyDeviceToHost, s));
        OVL_HIP(hipStreamSynchronize(s));
      }
      if (chiral && prev_worst_chiral > 0.0 && worst > 0.5 * prev_worst_chiral) {
        if (log_on()) fprintf(stderr, "[ovl cg] chiral cycle did not halve the residual: switching to D D^dag\n");
        chiral = false;
      }
      if (its >= maxiter || st->restarts >= opt.max_restarts) {
        rc = OVL_W_NOT_CONVERGED;
        break;
      }
      ++st->restarts;

      // chiral: per rhs the sector with the larger part of r,
      // ||P_+- r||^2 = (||r||^2 +- Re r^dag gamma5 r) / 2
      if (chiral) {
        blas_gamma5(OVL_F64, S.v64, r64.p, tmp64.p, R, s);
        S.rdot(r64.p, tmp64.p, OVL_F64, dS->pp, dS);
        std::vector<double> g5r(R);
        OVL_HIP(hipMemcpyAsync(g5r.data(), dS->pp, sizeof(double) * R, hipMemcpyDeviceToHost, s));
        OVL_HIP(hipStreamSynchronize(s));
        for (int r = 0; r < R; ++r) hS.sector[r] = g5r[r] >= 0.0 ? 1 : -1;
      }

      // inner system D e = r / scale, scale chosen so the rms element of the
      // scaled residual is O(1/8) (keeps FP16 iterates away from under/overflow)
      // adaptive precision: this cycle's inner sign is the coarsest whose
      // error, times the constant measured on the earlier cycles, stays
      // within the reduction that remains to reach tol (cycles that must
      // gain the full inner_tol keep the finest inner sign)
      if (ladder.size() > 1) {
        double need = 1.0;
        for (int r = 0; r < R; ++r) {
          const double rn = std::sqrt(rn2[r]);
          if (st->true_residual[r] > tol && rn > 0.0) need = std::min(need, 0.5 * tol * std::sqrt(bn2[r]) / rn);
        }
        int lv = 0;
        while (lv + 1 < static_cast<int>(ladder.size()) && k_sign * ladder[lv + 1]->delta <= need) ++lv;
        if (log_on() && lv != level)
          fprintf(stderr, "[ovl cg] cycle %d: inner sign n = %d (delta %.1e)\n", st->restarts,
                  static_cast<int>(ladder[lv]->c.size()) - 1, ladder[lv]->delta);
        set_level(lv);
        cycle_delta = ladder[lv]->delta;
      }
      for (int r = 0; r < R; ++r) {
        const double rn = std::sqrt(rn2[r]);
        const bool act = st->true_residual[r] > tol && rn > 0.0;
        const double sc = act ? rn / rms_target : 0.0;
        hS.scale[2 * r] = sc;
        hS.scale[2 * r + 1] = 0.0;
        hS.iscale[2 * r] = act ? 1.0 / sc : 0.0;
        hS.iscale[2 * r + 1] = 0.0;
        hS.active[r] = act ? 1 : 0;
        hS.bad[r] = 0;
        // relative stop of the inner solve: what remains to reach tol (with
        // margin) and, for a low-precision inner operator, inner_tol
        double rel = act ? 0.5 * tol * std::sqrt(bn2[r]) / rn : 1.0;
        if (P != OVL_F64) rel = std::max(rel, opt.inner_tol);
        rel = std::min(rel, 1.0);
        hS.target[r] = rel * rel * rms_target * rms_target;
      }
      OVL_HIP(hipMemcpyAsync(dS, &hS, sizeof(Scalars), hipMemcpyHostToDevice, s));
      OVL_HIP(hipStreamSynchronize(s));
      blas_axpby(OVL_F64, r64.p, dS->iscale, P, rin.p, nullptr, S.nsites, R, s);
      blas_zero(e64.p, S.v64 * R, s);
      if (chiral) {
        blas_chiral(P, S.vP, rin.p, R, dS->sector, s);
        S.norm2(rin.p, P, dS->rr, dS);
        blas_axpby(P, rin.p, dS->one, P, p.p, nullptr, S.nsites, R, s);
      } else {
        S.norm2(rin.p, P, dS->rr, dS);
        S.dm(p.p, rin.p, P, 1, true);
      }

      int inner = 0;
      for (;;) {
        int step;
        if (opt.graph_chunk > 0 && inner > 0 && !harvest) {
          hipGraphExec_t& gexec = gexecs[level];
          hipGraph_t& graph = graphs[level];
          if (gexec && (graph_chiral[level] != 0) != chiral) {
            OVL_HIP(hipGraphExecDestroy(gexec));
            OVL_HIP(hipGraphDestroy(graph));
            gexec = nullptr;
            graph = nullptr;
          }
          if (!gexec) {
            capturing = true;
            OVL_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
            const int64_t sa = st->sign_applies, da = st->dslash_applies;
            for (int k = 0; k < opt.graph_chunk; ++k) chiral ? body_chiral() : body();
            graph_chiral[level] = chiral ? 1 : 0;
            st->sign_applies = sa;  // captured, not executed: counted at replay
            st->dslash_applies = da;
            OVL_HIP(hipStreamEndCapture(s, &graph));
            capturing = false;
            OVL_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
          }
          OVL_HIP(hipGraphLaunch(gexec, s));
          step = opt.graph_chunk;
          const int sa_per_it = chiral ? 1 : 2;
          st->sign_applies += static_cast<int64_t>(sa_per_it) * R * step;
          st->dslash_applies += static_cast<int64_t>(sa_per_it) * R * step * S.per_sign_dw_in;
        } else {
          const int nrun = (opt.graph_chunk > 0 || harvest) ? 1 : check_every;
          for (int k = 0; k < nrun; ++k) chiral ? body_chiral() : body();
          step = nrun;
        }
        if (log_on() && (its + step) / 100 != its / 100)
          fprintf(stderr, "[ovl cg]   inner iteration %d\n", its + step);
        inner += step;
        its += step;
        OVL_HIP(hipMemcpyAsync(hS.active, dS->active, sizeof(hS.active) + sizeof(hS.bad), hipMemcpyDeviceToHost, s));
        OVL_HIP(hipStreamSynchronize(s));
        bool any = false, broke = false;
        for (int r = 0; r < R; ++r) {
          if (hS.bad[r] == 2 && !chiral) throw Error(OVL_E_NAN, "NaN or Inf in a CG iterate");
          if (hS.bad[r] == 1 && !chiral) throw Error(OVL_E_BREAKDOWN, "CG breakdown: p^dag p <= 0");
          broke = broke || hS.bad[r] != 0;
          any = any || hS.active[r];
        }
        if (broke) {
          chiral_failed = true;
          break;
        }
        if (!any || its >= maxiter) break;
      }
      if (chiral_failed) {
        // discard this cycle's correction and continue with D D^dag
        if (log_on()) fprintf(stderr, "[ovl cg] chiral sector operator not positive: switching to D D^dag\n");
        chiral = false;
        chiral_failed = false;
        continue;
      }
      if (chiral) {
        prev_worst_chiral = worst;
        // e = D(m)^dag y in FP64 (inner sign), into tmp64
        S.dm(tmp64.p, e64.p, OVL_F64, 1, true);
        blas_axpby(OVL_F64, tmp64.p, dS->scale, OVL_F64, x, dS->one, S.nsites, R, s);
      } else {
        // x += scale * e
        blas_axpby(OVL_F64, e64.p, dS->scale, OVL_F64, x, dS->one, S.nsites, R, s);
      }
    }
    st->iterations = its;
    OVL_HIP(hipStreamSynchronize(s));
  } catch (...) {
    drop_graphs();
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(ev);
    ws_retire_stream(s, us);
    (void)hipStreamDestroy(s);
    throw;
  }
  for (size_t k = 0; k < ladder.size(); ++k) {
    if (gexecs[k]) OVL_HIP(hipGraphExecDestroy(gexecs[k]));
    if (graphs[k]) OVL_HIP(hipGraphDestroy(graphs[k]));
  }
  // the caller's stream continues after the solve
  OVL_HIP(hipEventRecord(ev, s));
  OVL_HIP(hipStreamWaitEvent(us, ev, 0));
  OVL_HIP(hipStreamSynchronize(s));
  OVL_HIP(hipEventDestroy(ev));
  ws_retire_stream(s, us);
  OVL_HIP(hipStreamDestroy(s));
  st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return rc;
}


// ------------------------------------------------------------------- FGCR
// Flexible GCR with a right preconditioner M (the learned network, FP32) in
// the FP64 defect-correction loop.  The rhs of the batch run in lockstep:
// the bases W (the orthonormalised D(m) z) and Z (the matching search
// directions) of all rhs sit in two FP64 blocks, vector (i, r) at index
// i R + r, so one block_dot / block_axpy pair orthogonalises every rhs
// against its own earlier directions (the cross-rhs coefficients are set to
// zero on the device); M and D(m) run on the whole batch, and every Krylov
// scalar stays on the device.  The host reads the per-rhs flags once per
// iteration.
namespace {

// Device scalars of the batched GCR cycle, one slot per rhs.
struct GcrScalars {
  double rn2[OVL_MAX_RHS];           // ||r_r||^2 of the inner system
  double target2[OVL_MAX_RHS];       // rhs r stops once rn2 <= target2
  double tmp[2 * OVL_MAX_RHS];       // reduction output, (re, im) per rhs
  double dot[2 * OVL_MAX_RHS];       // W_{j,r}^dag r_r
  double alpha[2 * OVL_MAX_RHS];     // complex, 0 for inactive rhs
  double malpha[2 * OVL_MAX_RHS];
  double inv[2 * OVL_MAX_RHS];       // 1 / ||w_r|| (0 for inactive rhs)
  double one[2 * OVL_MAX_RHS];
  int active[OVL_MAX_RHS];
  int bad[OVL_MAX_RHS];              // 1: w = 0 or not finite, 2: residual not finite
};

// K[(i R + v) R + r] = -C[(i R + v) R + r] if v == r and rhs r is active, else 0:
// each rhs is projected on its own basis vectors only.
__global__ void gcr_coef_kernel(int n, int R, const double2* C, double2* K, const GcrScalars* S) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int r = k % R, v = (k / R) % R;
  const double2 c = C[k];
  K[k] = (v == r && S->active[r]) ? make_double2(-c.x, -c.y) : make_double2(0.0, 0.0);
}

__global__ void gcr_norm_kernel(int R, GcrScalars* S) {
  const int r = threadIdx.x;
  if (r >= R) return;
  double inv = 0.0;
  if (S->active[r]) {
    const double n2 = S->tmp[2 * r];
    if (n2 > 0.0 && n2 <= 1.79e308) {
      inv = 1.0 / sqrt(n2);
    } else {
      S->bad[r] = 1;
      S->active[r] = 0;
    }
  }
  S->inv[2 * r] = inv;
  S->inv[2 * r + 1] = 0.0;
}

__global__ void gcr_alpha_kernel(int R, GcrScalars* S) {
  const int r = threadIdx.x;
  if (r >= R) return;
  const bool a = S->active[r] != 0;
  const double re = a ? S->dot[2 * r] : 0.0, im = a ? S->dot[2 * r + 1] : 0.0;
  S->alpha[2 * r] = re;
  S->alpha[2 * r + 1] = im;
  S->malpha[2 * r] = -re;
  S->malpha[2 * r + 1] = -im;
}

__global__ void gcr_check_kernel(int R, GcrScalars* S) {
  const int r = threadIdx.x;
  if (r >= R || !S->active[r]) return;
  const double n2 = S->tmp[2 * r];
  S->rn2[r] = n2;
  if (!(n2 <= 1.79e308)) {
    S->bad[r] = 2;
    S->active[r] = 0;
  } else if (n2 <= S->target2[r]) {
    S->active[r] = 0;
  }
}

// dst_r = active_r ? inv_r src_r : 0 over R FP64 vectors of n16 elements
// (a select, so a non-finite src of an inactive rhs never reaches dst)
__global__ void gcr_store_kernel(size_t n16, size_t vs, const double2* src, double2* dst, const GcrScalars* S) {
  const int r = blockIdx.y;
  const size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (i >= n16) return;
  const size_t o = r * (vs / 16) + i;
  if (S->active[r]) {
    const double2 v = src[o];
    const double a = S->inv[2 * r];
    dst[o] = make_double2(a * v.x, a * v.y);
  } else {
    dst[o] = make_double2(0.0, 0.0);
  }
}

}  // namespace

int fgcr_solve(void* x, const void* b, int R, const ovl_gauge* u, double rho, double m, const ovl_sign* sg,
               const ovl_lowmodes* lm, const ovl_net* net, int restart, double tol, int maxiter,
               const ovl_solve_opts* o, ovl_solve_stats* st, hipStream_t us) {
  const auto t_start = std::chrono::steady_clock::now();
  const int P = o ? o->inner_prec : OVL_F64;
  const double inner_tol = o ? o->inner_tol : 0.0;
  const int max_restarts = o ? o->max_restarts : 50;
  check_prec(P);
  int recon = 0;
  (void)gauge_links(u, P, &recon);
  if (net) (void)gauge_links(u, OVL_F32, &recon);
  const ovl_geom* g = &u->geom;
  const size_t N = static_cast<size_t>(g->N);
  const size_t v64 = spinor_vec_bytes(g, OVL_F64), vP = spinor_vec_bytes(g, P), v32 = spinor_vec_bytes(g, OVL_F32);
  const int64_t per_sign_dw = 2 * (static_cast<int64_t>(sg->c.size()) - 1) + 1;
  const ovl_sign* sg_in = (o && o->inner_sign) ? o->inner_sign : sg;
  OVL_REQUIRE(sg_in->lam_max == sg->lam_max, OVL_E_ARG, "inner_sign must share lam_max with sign");
  const int64_t per_sign_dw_in = 2 * (static_cast<int64_t>(sg_in->c.size()) - 1) + 1;

  hipStream_t s;
  OVL_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipEvent_t ev;
  OVL_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  OVL_HIP(hipEventRecord(ev, us));
  OVL_HIP(hipStreamWaitEvent(s, ev, 0));
  // s now runs after everything queued on the caller's stream, so the free
  // workspace kept for that stream can serve this solve
  ws_retire_stream(us, s);
  int rc = OVL_OK;
  bool fallback = false;
  try {
    WsBuf r64(v64 * R, s), tmp64(v64 * R, s), e64(v64 * R, s), rin(v64 * R, s);
    WsBuf zP(vP * R, s), wP(vP * R, s), w64(v64 * R, s), z64(v64 * R, s);
    WsBuf r32(net ? v32 * R : 16, s), z32(net ? v32 * R : 16, s);
    WsBuf Wb(v64 * R * restart, s), Zb(v64 * R * restart, s);
    WsBuf sc(sizeof(double) * 4 * OVL_MAX_RHS, s);
    WsBuf gsb(sizeof(GcrScalars), s);
    WsBuf Cb(sizeof(double2) * static_cast<size_t>(restart) * R * R, s), Kb(sizeof(double2) * static_cast<size_t>(restart) * R * R, s);
    GcrScalars* dG = static_cast<GcrScalars*>(gsb.p);
    GcrScalars hG{};
    double* dsc = static_cast<double*>(sc.p);
    std::vector<double> bn2(R), rn2(R), h(4 * OVL_MAX_RHS);
    auto dev_scalars = [&](const std::vector<double>& v) {  // complex pairs -> dsc
      OVL_HIP(hipMemcpyAsync(dsc, v.data(), sizeof(double) * v.size(), hipMemcpyHostToDevice, s));
      OVL_HIP(hipStreamSynchronize(s));
    };
    auto norms = [&](const void* xx, int nr, size_t vs, int prec, std::vector<double>& out) {
      blas_norm2(prec, vs / 16, xx, nr, vs, dsc, s);
      OVL_HIP(hipMemcpyAsync(h.data(), dsc, sizeof(double) * 2 * nr, hipMemcpyDeviceToHost, s));
      OVL_HIP(hipStreamSynchronize(s));
      out.resize(nr);
      for (int r = 0; r < nr; ++r) out[r] = h[2 * r];
    };
    auto dm = [&](void* out, const void* in, int prec, bool inner) {
      overlap_apply(out, in, u, rho, m, inner ? sg_in : sg, lm, 1, prec, R, s);
      st->sign_applies += R;
      st->dslash_applies += R * (inner ? per_sign_dw_in : per_sign_dw);
    };
    auto blk = [&](void* base, int j) { return static_cast<char*>(base) + static_cast<size_t>(j) * R * v64; };
    const size_t n16 = v64 / 16;
    const dim3 sgrid((n16 + 255) / 256, R);

    norms(b, R, v64, OVL_F64, bn2);
    for (int r = 0; r < R; ++r) OVL_REQUIRE(std::isfinite(bn2[r]), OVL_E_NAN, "right-hand side contains NaN or Inf");
    const double rms_target = P == OVL_F64 ? 1.0 : std::sqrt(12.0 * N) / 8.0;
    int its = 0;
    st->restarts = 0;
    for (int r = 0; r < OVL_MAX_RHS; ++r) {
      hG.one[2 * r] = 1.0;
      hG.one[2 * r + 1] = 0.0;
    }
    for (;;) {
      dm(tmp64.p, x, OVL_F64, false);
      std::vector<double> c(4 * OVL_MAX_RHS, 0.0);
      for (int r = 0; r < R; ++r) {
        c[2 * r] = 1.0;
        c[2 * OVL_MAX_RHS + 2 * r] = -1.0;
      }
      dev_scalars(c);
      blas_axpby(OVL_F64, b, dsc, OVL_F64, r64.p, nullptr, N, R, s);
      blas_axpby(OVL_F64, tmp64.p, dsc + 2 * OVL_MAX_RHS, OVL_F64, r64.p, dsc, N, R, s);
      norms(r64.p, R, v64, OVL_F64, rn2);
      bool done = true;
      std::vector<int> active(R);
      for (int r = 0; r < R; ++r) {
        const double res = bn2[r] > 0 ? std::sqrt(rn2[r] / bn2[r]) : 0.0;
        OVL_REQUIRE(std::isfinite(res), OVL_E_NAN, "true residual is NaN or Inf");
        st->true_residual[r] = res;
        active[r] = res > tol;
        if (active[r]) done = false;
      }
      if (log_on()) {
        double worst = 0.0;
        for (int r = 0; r < R; ++r) worst = std::max(worst, st->true_residual[r]);
        fprintf(stderr, "[ovl fgcr] cycle %d: %d iterations, max FP64 true residual %.3e\n", st->restarts, its, worst);
      }
      if (done) break;
      if (its >= maxiter || st->restarts >= max_restarts) {
        rc = OVL_W_NOT_CONVERGED;
        break;
      }
      ++st->restarts;
      // scaled inner system D e = r / scale
      std::vector<double> scale(R), isc(2 * OVL_MAX_RHS, 0.0);
      for (int r = 0; r < R; ++r) {
        const double rn = std::sqrt(rn2[r]);
        scale[r] = active[r] ? rn / rms_target : 0.0;
        isc[2 * r] = active[r] ? 1.0 / scale[r] : 0.0;
        double rel = active[r] ? 0.5 * tol * std::sqrt(bn2[r]) / rn : 1.0;
        if (P != OVL_F64) rel = std::max(rel, inner_tol);
        const double tg = std::min(rel, 1.0) * rms_target;
        hG.target2[r] = tg * tg;
        hG.rn2[r] = active[r] ? rms_target * rms_target : 0.0;
        hG.active[r] = active[r];
        hG.bad[r] = 0;
      }
      dev_scalars(isc);
      blas_axpby(OVL_F64, r64.p, dsc, OVL_F64, rin.p, nullptr, N, R, s);
      blas_zero(e64.p, v64 * R, s);
      OVL_HIP(hipMemcpyAsync(dG, &hG, sizeof(GcrScalars), hipMemcpyHostToDevice, s));
      bool inner_done = false;
      while (!inner_done && its < maxiter) {
        std::vector<double> cycle_start(hG.rn2, hG.rn2 + R);
        int j = 0;
        bool any = true;
        for (; j < restart && its < maxiter; ++j) {
          // z = M r (FP32 network) or z = r, then w = D(m) z at the inner precision
          if (net) {
            blas_convert(OVL_F64, rin.p, OVL_F32, r32.p, N, R, s);
            net_apply(net, u, r32.p, z32.p, R, s);
            blas_convert(OVL_F32, z32.p, P, zP.p, N, R, s);
          } else {
            blas_convert(OVL_F64, rin.p, P, zP.p, N, R, s);
          }
          dm(wP.p, zP.p, P, true);
          blas_convert(P, wP.p, OVL_F64, w64.p, N, R, s);
          blas_convert(P, zP.p, OVL_F64, z64.p, N, R, s);
          ++its;
          // w, z -= (own earlier directions) (W^dag w), twice
          const int nb = j * R;
          for (int pass = 0; pass < (j > 0 ? 2 : 0); ++pass) {
            block_dot(g, Wb.p, nb, w64.p, OVL_F64, R, static_cast<double2*>(Cb.p), s);
            hipLaunchKernelGGL(gcr_coef_kernel, dim3((nb * R + 255) / 256), dim3(256), 0, s, nb * R, R,
                               static_cast<const double2*>(Cb.p), static_cast<double2*>(Kb.p), dG);
            block_axpy(g, Wb.p, nb, static_cast<const double2*>(Kb.p), w64.p, OVL_F64, R, true, s);
            block_axpy(g, Zb.p, nb, static_cast<const double2*>(Kb.p), z64.p, OVL_F64, R, true, s);
          }
          // W_j = w / ||w||, Z_j = z / ||w||
          blas_norm2(OVL_F64, n16, w64.p, R, v64, dG->tmp, s);
          hipLaunchKernelGGL(gcr_norm_kernel, dim3(1), dim3(64), 0, s, R, dG);
          hipLaunchKernelGGL(gcr_store_kernel, sgrid, dim3(256), 0, s, n16, v64,
                             static_cast<const double2*>(w64.p), reinterpret_cast<double2*>(blk(Wb.p, j)), dG);
          hipLaunchKernelGGL(gcr_store_kernel, sgrid, dim3(256), 0, s, n16, v64,
                             static_cast<const double2*>(z64.p), reinterpret_cast<double2*>(blk(Zb.p, j)), dG);
          // alpha = W_j^dag r; e += alpha Z_j; r -= alpha W_j
          blas_dot(OVL_F64, n16, blk(Wb.p, j), rin.p, R, v64, dG->dot, s);
          hipLaunchKernelGGL(gcr_alpha_kernel, dim3(1), dim3(64), 0, s, R, dG);
          blas_axpby(OVL_F64, blk(Zb.p, j), dG->alpha, OVL_F64, e64.p, dG->one, N, R, s);
          blas_axpby(OVL_F64, blk(Wb.p, j), dG->malpha, OVL_F64, rin.p, dG->one, N, R, s);
          blas_norm2(OVL_F64, n16, rin.p, R, v64, dG->tmp, s);
          hipLaunchKernelGGL(gcr_check_kernel, dim3(1), dim3(64), 0, s, R, dG);
          OVL_HIP(hipGetLastError());
          OVL_HIP(hipMemcpyAsync(&hG, dG, sizeof(GcrScalars), hipMemcpyDeviceToHost, s));
          OVL_HIP(hipStreamSynchronize(s));
          any = false;
          for (int r = 0; r < R; ++r) {
            if (hG.bad[r]) fallback = true;
            any = any || hG.active[r];
          }
          if (fallback || !any) break;
        }
        if (fallback) break;
        bool stagnant = false;
        for (int r = 0; r < R; ++r)
          if (hG.active[r] && j >= restart && hG.rn2[r] > 0.81 * cycle_start[r]) stagnant = true;
        if (stagnant) fallback = true;
        inner_done = !any || fallback;
      }
      // x += scale * e
      std::vector<double> scv(4 * OVL_MAX_RHS, 0.0);
      for (int r = 0; r < R; ++r) {
        scv[2 * r] = scale[r];
        scv[2 * OVL_MAX_RHS + 2 * r] = 1.0;
      }
      dev_scalars(scv);
      blas_axpby(OVL_F64, e64.p, dsc, OVL_F64, x, dsc + 2 * OVL_MAX_RHS, N, R, s);
      OVL_HIP(hipStreamSynchronize(s));
      if (fallback) break;
    }
    st->iterations = its;
  } catch (...) {
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(ev);
    ws_retire_stream(s, us);
    (void)hipStreamDestroy(s);
    throw;
  }
  OVL_HIP(hipEventRecord(ev, s));
  OVL_HIP(hipStreamWaitEvent(us, ev, 0));
  OVL_HIP(hipStreamSynchronize(s));
  OVL_HIP(hipEventDestroy(ev));
  ws_retire_stream(s, us);
  OVL_HIP(hipStreamDestroy(s));
  if (fallback) {
    // plain CG finishes the solve from the current x
    ovl_solve_stats cs{};
    ovl_solve_opts co{};
    co.inner_prec = static_cast<ovl_prec>(P);
    co.inner_tol = inner_tol;
    co.graph_chunk = o ? o->graph_chunk : 0;
    co.check_every = 1;
    co.max_restarts = max_restarts;
    co.inner_sign = o ? o->inner_sign : nullptr;
    const int its0 = st->iterations;
    const int64_t sa = st->sign_applies, da = st->dslash_applies;
    rc = cg_solve(x, b, R, u, rho, m, sg, lm, tol, std::max(0, maxiter - its0), &co, &cs, us);
    *st = cs;
    st->iterations += its0;
    st->sign_applies += sa;
    st->dslash_applies += da;
    st->fallback_used = 1;
  }
  st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return rc;
}

// Multi-mass CG (eq. 3 and 8).  When sign^2 = 1,
//   D(m) D(m)^dag = c(m) (K + sigma(m)),  K = gamma5 sign + sign gamma5,
//   c(m) = rho^2 - m^2/4,  sigma(m) = (2 rho^2 + m^2/2) / c(m),
// so every mass is a shift of one Hermitian operator.  Stage 1 runs CG on
// K + sigma_0 (sigma_0 the smallest shift: the lightest mass) and gets the
// other shifted solutions y_j from the same Krylov space through the
// shifted-CG recurrences (zeta_j), at the inner precision and to the inner
// tolerance.  Then x_j = D(m_j)^dag y_j / c_j, and each x_j goes through
// the FP64 defect-correction loop of cg_solve (which also absorbs the O(delta)
// difference between D D^dag and c (K + sigma) of the polynomial sign).
namespace {

constexpr int MM_MAX = 8;  // masses

// Device scalars of the shifted CG stage, one slot per (mass, rhs).
struct MMScalars {
  double zeta[MM_MAX][OVL_MAX_RHS], zeta_p[MM_MAX][OVL_MAX_RHS], zn[MM_MAX][OVL_MAX_RHS];
  double alpha_j[MM_MAX][OVL_MAX_RHS];
  double coef[MM_MAX][OVL_MAX_RHS][4];  // alpha_j, zeta_next, beta_j, active (for the fused update)
  double sig[MM_MAX];                   // sigma_j - sigma_base
  double alpha_p[OVL_MAX_RHS], beta_p[OVL_MAX_RHS], rr[OVL_MAX_RHS], bn2[OVL_MAX_RHS];
  double alpha[OVL_MAX_RHS];
  double dot[2 * OVL_MAX_RHS];   // reduction outputs, (re, im) per rhs
  double nrm[2 * OVL_MAX_RHS];
  double malpha[2 * OVL_MAX_RHS];  // (-alpha, 0) per rhs
  double one[2 * OVL_MAX_RHS];
  double rel;
  int act[MM_MAX][OVL_MAX_RHS];
  int live[OVL_MAX_RHS];
  int bad[OVL_MAX_RHS];  // 1 breakdown (p^dag A p <= 0), 2 NaN/Inf
};

// alpha = rr / p^dag A p per live rhs, and every shift's step alpha_j from
// the zeta recurrence (Jegerlehner); one thread per rhs.
__global__ void mm_alpha_kernel(int R, int nm, int base, MMScalars* S) {
  const int r = threadIdx.x;
  if (r >= R) return;
  double a = 0.0;
  if (S->live[r]) {
    const double pq = S->dot[2 * r];
    if (!(pq == pq) || isinf(pq)) {
      S->bad[r] = 2;
      S->live[r] = 0;
    } else if (pq <= 0.0) {
      S->bad[r] = 1;
      S->live[r] = 0;
    } else {
      a = S->rr[r] / pq;
    }
  }
  S->alpha[r] = a;
  S->malpha[2 * r] = -a;
  S->malpha[2 * r + 1] = 0.0;
  for (int j = 0; j < nm; ++j) {
    double z = 1.0, aj = a;
    if (j != base && S->live[r]) {
      const double zc = S->zeta[j][r], zp = S->zeta_p[j][r];
      const double den = a * S->beta_p[r] * (zp - zc) + zp * S->alpha_p[r] * (1.0 + S->sig[j] * a);
      z = den != 0.0 ? zc * zp * S->alpha_p[r] / den : 0.0;
      aj = zc != 0.0 ? a * z / zc : 0.0;
    }
    S->zn[j][r] = S->live[r] ? z : S->zeta[j][r];
    S->alpha_j[j][r] = (S->live[r] && S->act[j][r]) ? aj : 0.0;
  }
}

// beta from the new residual, the fused-update coefficients, then the
// shifted state for the next iteration and the convergence of each shift
// (its residual is zeta_j r).
__global__ void mm_beta_kernel(int R, int nm, MMScalars* S) {
  const int r = threadIdx.x;
  if (r >= R) return;
  const double rrn = S->nrm[2 * r];
  const bool live = S->live[r] != 0;
  if (live && (!(rrn == rrn) || isinf(rrn))) {
    S->bad[r] = 2;
    S->live[r] = 0;
  }
  const bool ok = S->live[r] != 0;
  const double beta = ok ? rrn / S->rr[r] : 0.0;
  int any = 0;
  for (int j = 0; j < nm; ++j) {
    const bool on = ok && S->act[j][r];
    const double zc = S->zeta[j][r], zn = S->zn[j][r];
    const double ratio = (zc != 0.0) ? zn / zc : 0.0;
    S->coef[j][r][0] = S->alpha_j[j][r];
    S->coef[j][r][1] = on ? zn : 0.0;
    S->coef[j][r][2] = on ? beta * ratio * ratio : 1.0;
    S->coef[j][r][3] = on ? 1.0 : 0.0;
    if (ok) {
      S->zeta_p[j][r] = zc;
      S->zeta[j][r] = zn;
      if (S->act[j][r] && fabs(zn) * sqrt(rrn) <= S->rel * sqrt(S->bn2[r])) S->act[j][r] = 0;
    }
    any |= S->act[j][r];
  }
  if (ok) {
    S->alpha_p[r] = S->alpha[r];
    S->beta_p[r] = beta;
    S->rr[r] = rrn;
    S->live[r] = any;
  }
}

// For every FP64 element of rhs r (blockIdx.y) and every shift j with its
// coefficient row active: y_j += alpha_j p_j, then p_j = zeta_j r + beta_j p_j
// (the base residual is read once for all shifts).
__global__ void mm_update_kernel(size_t n16, int R, int nm, const double2* __restrict__ res, double2* Y, double2* Pj,
                                 const MMScalars* S) {
  const int r = blockIdx.y;
  const size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (e >= n16) return;
  const double2 rv = res[r * n16 + e];
  for (int j = 0; j < nm; ++j) {
    const double* c = S->coef[j][r];
    if (c[3] == 0.0 && c[0] == 0.0) continue;
    const size_t o = (static_cast<size_t>(j) * R + r) * n16 + e;
    const double2 pv = Pj[o];
    double2 yv = Y[o];
    yv.x = fma(c[0], pv.x, yv.x);
    yv.y = fma(c[0], pv.y, yv.y);
    Y[o] = yv;
    if (c[3] != 0.0) Pj[o] = make_double2(fma(c[1], rv.x, c[2] * pv.x), fma(c[1], rv.y, c[2] * pv.y));
  }
}

}  // namespace

int cg_multimass(void* const* xs, const void* b, int R, const ovl_gauge* u, double rho, const double* masses, int nm,
                 const ovl_sign* sg, const ovl_lowmodes* lm, double tol, int maxiter, const ovl_solve_opts* o,
                 ovl_solve_stats* sts, hipStream_t us) {
  const auto t_start = std::chrono::steady_clock::now();
  const int P = o ? o->inner_prec : OVL_F64;
  check_prec(P);
  const double inner_tol = o ? o->inner_tol : 0.0;
  const ovl_sign* sg_in = (o && o->inner_sign) ? o->inner_sign : sg;
  OVL_REQUIRE(sg_in->lam_max == sg->lam_max, OVL_E_ARG, "inner_sign must share lam_max with sign");
  int recon = 0;
  (void)gauge_links(u, P, &recon);
  const ovl_geom* g = &u->geom;
  const size_t N = static_cast<size_t>(g->N);
  const size_t v64 = spinor_vec_bytes(g, OVL_F64), vP = spinor_vec_bytes(g, P);
  const int64_t per_sign_dw_in = 2 * (static_cast<int64_t>(sg_in->c.size()) - 1) + 1;
  std::vector<double> c(nm), sigma(nm);
  int base = 0;
  for (int j = 0; j < nm; ++j) {
    c[j] = rho * rho - 0.25 * masses[j] * masses[j];
    sigma[j] = (2.0 * rho * rho + 0.5 * masses[j] * masses[j]) / c[j];
    if (sigma[j] < sigma[base]) base = j;
  }
  for (int j = 0; j < nm; ++j) sts[j] = ovl_solve_stats{};
  ovl_solve_stats& s0 = sts[base];

  hipStream_t s;
  OVL_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipEvent_t ev;
  OVL_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  OVL_HIP(hipEventRecord(ev, us));
  OVL_HIP(hipStreamWaitEvent(s, ev, 0));
  // s now runs after everything queued on the caller's stream, so the free
  // workspace kept for that stream can serve this solve
  ws_retire_stream(us, s);
  int its = 0;
  try {
    WsBuf r64(v64 * R, s), q64(v64 * R, s), t64(v64 * R, s), pP(vP * R, s), qP(vP * R, s), tP(vP * R, s);
    WsBuf pj(v64 * R * nm, s), yj(v64 * R * nm, s);
    WsBuf sc(sizeof(double) * 2 * OVL_MAX_RHS * 4, s);
    double* dsc = static_cast<double*>(sc.p);
    auto vec = [&](void* base_, int j) { return static_cast<char*>(base_) + static_cast<size_t>(j) * v64 * R; };
    std::vector<double> hbuf(2 * OVL_MAX_RHS * 4, 0.0);
    // four per-rhs complex coefficient rows on the device
    auto upload = [&](const std::vector<double>& a0, const std::vector<double>& a1, const std::vector<double>& a2,
                      const std::vector<double>& a3) {
      std::fill(hbuf.begin(), hbuf.end(), 0.0);
      for (int r = 0; r < R; ++r) {
        hbuf[2 * r] = a0[r];
        hbuf[2 * OVL_MAX_RHS + 2 * r] = a1[r];
        hbuf[4 * OVL_MAX_RHS + 2 * r] = a2[r];
        hbuf[6 * OVL_MAX_RHS + 2 * r] = a3[r];
      }
      OVL_HIP(hipMemcpyAsync(dsc, hbuf.data(), sizeof(double) * hbuf.size(), hipMemcpyHostToDevice, s));
      OVL_HIP(hipStreamSynchronize(s));
    };
    const double* A0 = dsc;
    const double* A1 = dsc + 2 * OVL_MAX_RHS;
    const double* A2 = dsc + 4 * OVL_MAX_RHS;
    const double* A3 = dsc + 6 * OVL_MAX_RHS;
    WsBuf red(sizeof(double) * 2 * OVL_MAX_RHS, s);
    auto reduce = [&](const void* x1, const void* x2) {  // Re x1^dag x2 per rhs (x2 null: norm^2)
      if (x2)
        blas_dot(OVL_F64, v64 / 16, x1, x2, R, v64, static_cast<double*>(red.p), s);
      else
        blas_norm2(OVL_F64, v64 / 16, x1, R, v64, static_cast<double*>(red.p), s);
      std::vector<double> h(2 * R);
      OVL_HIP(hipMemcpyAsync(h.data(), red.p, sizeof(double) * 2 * R, hipMemcpyDeviceToHost, s));
      OVL_HIP(hipStreamSynchronize(s));
      std::vector<double> out(R);
      for (int r = 0; r < R; ++r) out[r] = h[2 * r];
      return out;
    };
    const std::vector<double> ones(R, 1.0), zeros(R, 0.0);
    // r = b, p_j = b, y_j = 0
    upload(ones, zeros, zeros, zeros);
    blas_axpby(OVL_F64, b, A0, OVL_F64, r64.p, nullptr, N, R, s);
    for (int j = 0; j < nm; ++j) {
      blas_axpby(OVL_F64, b, A0, OVL_F64, vec(pj.p, j), nullptr, N, R, s);
      blas_zero(vec(yj.p, j), v64 * R, s);
    }
    const std::vector<double> bn2 = reduce(b, nullptr);
    for (int r = 0; r < R; ++r) OVL_REQUIRE(std::isfinite(bn2[r]), OVL_E_NAN, "right-hand side contains NaN or Inf");
    // the shifted state lives on the device; the host reads the flags once
    // per iteration
    WsBuf mmb(sizeof(MMScalars), s);
    MMScalars* dM = static_cast<MMScalars*>(mmb.p);
    MMScalars hM{};
    hM.rel = std::max(0.5 * tol, P == OVL_F64 ? 0.0 : inner_tol);
    for (int j = 0; j < nm; ++j) hM.sig[j] = sigma[j] - sigma[base];
    for (int r = 0; r < R; ++r) {
      hM.rr[r] = bn2[r];
      hM.bn2[r] = bn2[r];
      hM.alpha_p[r] = 1.0;
      hM.beta_p[r] = 0.0;
      hM.one[2 * r] = 1.0;
      hM.live[r] = bn2[r] > 0.0;
      for (int j = 0; j < nm; ++j) {
        hM.zeta[j][r] = hM.zeta_p[j][r] = 1.0;
        hM.act[j][r] = bn2[r] > 0.0;
      }
    }
    OVL_HIP(hipMemcpyAsync(dM, &hM, sizeof(MMScalars), hipMemcpyHostToDevice, s));
    upload(ones, ones, zeros, zeros);  // A0 = A1 = 1 for the q assembly, for the whole stage
    const size_t n16 = v64 / 16;
    int live_flags[2 * OVL_MAX_RHS];
    while (its < maxiter) {
      OVL_HIP(hipMemcpyAsync(live_flags, dM->live, sizeof(int) * 2 * OVL_MAX_RHS, hipMemcpyDeviceToHost, s));
      OVL_HIP(hipStreamSynchronize(s));  // live and bad are adjacent
      bool any = false;
      for (int r = 0; r < R; ++r) {
        if (live_flags[OVL_MAX_RHS + r] == 2) throw Error(OVL_E_NAN, "NaN or Inf in a multi-mass CG iterate");
        if (live_flags[OVL_MAX_RHS + r] == 1) throw Error(OVL_E_BREAKDOWN, "multi-mass CG breakdown: p^dag A p <= 0");
        any = any || live_flags[r];
      }
      if (!any) break;
      // q = (K + sigma_0) p_0 at the inner precision
      void* p0 = vec(pj.p, base);
      blas_convert(OVL_F64, p0, P, pP.p, N, R, s);
      overlap_combine(qP.p, pP.p, u, rho, sigma[base], 1.0, sg_in, lm, P, R, s);
      overlap_combine_dag(tP.p, pP.p, u, rho, 0.0, 1.0, sg_in, lm, P, R, s);
      blas_convert(P, qP.p, OVL_F64, q64.p, N, R, s);
      blas_convert(P, tP.p, OVL_F64, t64.p, N, R, s);
      blas_axpby(OVL_F64, t64.p, A0, OVL_F64, q64.p, A1, N, R, s);
      s0.sign_applies += 2 * R;
      s0.dslash_applies += 2 * R * per_sign_dw_in;
      blas_dot(OVL_F64, n16, p0, q64.p, R, v64, dM->dot, s);
      hipLaunchKernelGGL(mm_alpha_kernel, dim3(1), dim3(64), 0, s, R, nm, base, dM);
      // r -= alpha q
      blas_axpby(OVL_F64, q64.p, dM->malpha, OVL_F64, r64.p, dM->one, N, R, s);
      blas_norm2(OVL_F64, n16, r64.p, R, v64, dM->nrm, s);
      hipLaunchKernelGGL(mm_beta_kernel, dim3(1), dim3(64), 0, s, R, nm, dM);
      // y_j += alpha_j p_j;  p_j = zeta_j r + beta_j p_j
      hipLaunchKernelGGL(mm_update_kernel, dim3((n16 + 255) / 256, R), dim3(256), 0, s, n16, R, nm,
                         static_cast<const double2*>(r64.p), static_cast<double2*>(yj.p),
                         static_cast<double2*>(pj.p), dM);
      OVL_HIP(hipGetLastError());
      ++its;
      if (log_on() && its % 100 == 0) fprintf(stderr, "[ovl multimass] iteration %d\n", its);
    }
    // x_j = D(m_j)^dag y_j / c_j in FP64
    for (int j = 0; j < nm; ++j) {
      overlap_apply(t64.p, vec(yj.p, j), u, rho, masses[j], sg, lm, 2, OVL_F64, R, s);
      std::vector<double> ic(R, 1.0 / c[j]);
      upload(ic, zeros, zeros, zeros);
      blas_axpby(OVL_F64, t64.p, A0, OVL_F64, xs[j], nullptr, N, R, s);
    }
    OVL_HIP(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(ev);
    ws_retire_stream(s, us);
    (void)hipStreamDestroy(s);
    throw;
  }
  OVL_HIP(hipEventRecord(ev, s));
  OVL_HIP(hipStreamWaitEvent(us, ev, 0));
  OVL_HIP(hipStreamSynchronize(s));
  OVL_HIP(hipEventDestroy(ev));
  ws_retire_stream(s, us);
  OVL_HIP(hipStreamDestroy(s));
  const double t_shift = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  if (log_on()) fprintf(stderr, "[ovl multimass] shifted CG: %d iterations, %.2f s\n", its, t_shift);
  // FP64 defect correction per mass from x_j
  int rc = OVL_OK;
  for (int j = 0; j < nm; ++j) {
    ovl_solve_stats cs{};
    const int r_j = cg_solve(xs[j], b, R, u, rho, masses[j], sg, lm, tol, std::max(0, maxiter - its), o, &cs, us);
    if (r_j != OVL_OK) rc = r_j;
    const int64_t sa = sts[j].sign_applies, da = sts[j].dslash_applies;
    sts[j] = cs;
    sts[j].sign_applies += sa;
    sts[j].dslash_applies += da;
  }
  sts[base].iterations += its;
  sts[base].seconds += t_shift;
  return rc;
}

}  // namespace ovl

using namespace ovl;

extern "C" {

int ovl_cg_solve(void* x, const void* b, int nrhs, const ovl_gauge* u, double rho, double m, const ovl_sign* sign,
                 const ovl_lowmodes* lowmodes, double tol, int maxiter, const ovl_solve_opts* opts,
                 ovl_solve_stats* stats, ovl_stream_t s) {
  return guard([&] {
    OVL_REQUIRE(x && b && u && sign && stats, OVL_E_ARG, "null argument");
    OVL_REQUIRE(nrhs >= 1 && nrhs <= OVL_MAX_RHS, OVL_E_ARG, "cg_solve: 1 <= nrhs <= 12");
    OVL_REQUIRE(x != b, OVL_E_ALIAS, "x must not alias b");
    OVL_REQUIRE(tol > 0.0 && maxiter >= 0, OVL_E_ARG, "need tol > 0 and maxiter >= 0");
    OVL_REQUIRE(m > -2.0 * rho && m < 2.0 * rho, OVL_E_ARG, "need |m| < 2 rho");
    if (lowmodes && lowmodes->ell == 0) lowmodes = nullptr;
    if (opts) OVL_REQUIRE(opts->graph_chunk >= 0 && opts->graph_chunk <= 1000, OVL_E_ARG, "graph_chunk out of range");
    *stats = ovl_solve_stats{};
    return cg_solve(x, b, nrhs, u, rho, m, sign, lowmodes, tol, maxiter, opts, stats, static_cast<hipStream_t>(s));
  });
}

int ovl_fgcr_solve(void* x, const void* b, int nrhs, const ovl_gauge* u, double rho, double m, const ovl_sign* sign,
                   const ovl_lowmodes* lowmodes, const ovl_net* M, int restart, double tol, int maxiter,
                   const ovl_solve_opts* opts, ovl_solve_stats* stats, ovl_stream_t s) {
  return guard([&] {
    OVL_REQUIRE(x && b && u && sign && stats, OVL_E_ARG, "null argument");
    OVL_REQUIRE(nrhs >= 1 && nrhs <= OVL_MAX_RHS, OVL_E_ARG, "fgcr_solve: 1 <= nrhs <= 12");
    OVL_REQUIRE(restart >= 1 && restart <= 32, OVL_E_ARG, "fgcr_solve: 1 <= restart <= 32");
    OVL_REQUIRE(x != b, OVL_E_ALIAS, "x must not alias b");
    OVL_REQUIRE(tol > 0.0 && maxiter >= 0, OVL_E_ARG, "need tol > 0 and maxiter >= 0");
    if (lowmodes && lowmodes->ell == 0) lowmodes = nullptr;
    *stats = ovl_solve_stats{};
    return fgcr_solve(x, b, nrhs, u, rho, m, sign, lowmodes, M, restart, tol, maxiter, opts, stats,
                      static_cast<hipStream_t>(s));
  });
}

int ovl_cg_multimass(void* const* x, const void* b, int nrhs, const ovl_gauge* u, double rho, const double* masses,
                     int nmass, const ovl_sign* sign, const ovl_lowmodes* lowmodes, double tol, int maxiter,
                     const ovl_solve_opts* opts, ovl_solve_stats* stats, ovl_stream_t s) {
  return guard([&] {
    OVL_REQUIRE(x && b && u && sign && stats && masses, OVL_E_ARG, "null argument");
    OVL_REQUIRE(nmass >= 1 && nmass <= 8, OVL_E_ARG, "cg_multimass: 1 <= nmass <= 8");
    OVL_REQUIRE(nrhs >= 1 && nrhs <= OVL_MAX_RHS, OVL_E_ARG, "cg_multimass: 1 <= nrhs <= 12");
    OVL_REQUIRE(tol > 0.0 && maxiter >= 0, OVL_E_ARG, "need tol > 0 and maxiter >= 0");
    for (int j = 0; j < nmass; ++j) {
      OVL_REQUIRE(x[j] && x[j] != b, OVL_E_ALIAS, "each x_j must be a separate buffer, not b");
      for (int k = 0; k < j; ++k) OVL_REQUIRE(x[k] != x[j], OVL_E_ALIAS, "x buffers must differ");
      OVL_REQUIRE(masses[j] > -2.0 * rho && masses[j] < 2.0 * rho, OVL_E_ARG, "need |m| < 2 rho");
    }
    OVL_REQUIRE(!(opts && opts->chiral), OVL_E_ARG, "cg_multimass: chiral mode not supported");
    OVL_REQUIRE(!(opts && opts->harvest_x && opts->harvest_b && opts->harvest_cap > 0), OVL_E_ARG,
                "cg_multimass: no harvesting");
    if (lowmodes && lowmodes->ell == 0) lowmodes = nullptr;
    return cg_multimass(x, b, nrhs, u, rho, masses, nmass, sign, lowmodes, tol, maxiter, opts, stats,
                        static_cast<hipStream_t>(s));
  });
}

int ovl_propagator(void* out, const void* x, const ovl_gauge* u, double rho, const ovl_sign* sign,
                   const ovl_lowmodes* lowmodes, ovl_prec prec, int nrhs, ovl_stream_t s) {
  return guard([&] {
    OVL_REQUIRE(out && x && u && sign, OVL_E_ARG, "null argument");
    check_prec(prec);
    check_nrhs(nrhs);
    OVL_REQUIRE(out != x, OVL_E_ALIAS, "output must not alias the input");
    if (lowmodes && lowmodes->ell == 0) lowmodes = nullptr;
    // (1 - D/2) x = x/2 - gamma5 sign(H_w) x / 2
    overlap_combine(out, x, u, rho, 0.5, -0.5, sign, lowmodes, prec, nrhs, static_cast<hipStream_t>(s));
    return OVL_OK;
  });
}

}  // extern "C"
