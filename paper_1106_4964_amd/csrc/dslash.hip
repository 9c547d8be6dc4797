// Wilson hopping stencil (arXiv:1106.4964 Sec. II, eq. 1-2) with fused
// epilogues, for every storage precision and link representation.
//
// One thread computes the 12 complex output components of one site.  For
// each of the 8 directions it loads the neighbour spinor, spin-projects it
// to a 2x3 half spinor with (1 -+ gamma_mu), multiplies both colour vectors
// by U_mu(x) or U_mu(x-mu)^dag and adds the result back, the lower two spin
// components being fixed multiples of the upper two (chiral basis).
// The epilogue forms  G(a*in + b*hop) + sum_j c_j G_j(v_j)  at the output
// site, which covers D_w(m), H_w = gamma5 D_w(-rho), and the Clenshaw
// update of the polynomial sign function (Sec. V) in one pass.
#include "ops.h"

namespace ovl {
namespace {

// Half-spinor projection (1 + SGN*gamma_mu) psi -> h[2][3] and the
// reconstruction of the lower spin components from U*h.  Chiral basis:
//   mu=0: (1-g1): h0=s0+i s3, h1=s1+i s2, lower=(-i h1,-i h0); (1+g1): signs of i flip
//   mu=1: (1-g2): h0=s0+s3,   h1=s1-s2,   lower=(-h1, h0);     (1+g2): h0=s0-s3, h1=s1+s2, lower=(h1,-h0)
//   mu=2: (1-g3): h0=s0+i s2, h1=s1-i s3, lower=(-i h0, i h1); (1+g3): signs of i flip
//   mu=3: (1-g4): h0=s0-s2,   h1=s1-s3,   lower=(-h0,-h1);     (1+g4): h0=s0+s2, h1=s1+s3, lower=(h0,h1)
template <int MU, int SGN, typename T>
__device__ inline void project(const Cx<T>* s, Cx<T> (*h)[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const Cx<T> s0 = s[c], s1 = s[3 + c], s2 = s[6 + c], s3 = s[9 + c];
    if constexpr (MU == 0) {
      if constexpr (SGN < 0) {
        h[0][c] = s0 + times_i(s3);
        h[1][c] = s1 + times_i(s2);
      } else {
        h[0][c] = s0 - times_i(s3);
        h[1][c] = s1 - times_i(s2);
      }
    } else if constexpr (MU == 1) {
      if constexpr (SGN < 0) {
        h[0][c] = s0 + s3;
        h[1][c] = s1 - s2;
      } else {
        h[0][c] = s0 - s3;
        h[1][c] = s1 + s2;
      }
    } else if constexpr (MU == 2) {
      if constexpr (SGN < 0) {
        h[0][c] = s0 + times_i(s2);
        h[1][c] = s1 - times_i(s3);
      } else {
        h[0][c] = s0 - times_i(s2);
        h[1][c] = s1 + times_i(s3);
      }
    } else {
      if constexpr (SGN < 0) {
        h[0][c] = s0 - s2;
        h[1][c] = s1 - s3;
      } else {
        h[0][c] = s0 + s2;
        h[1][c] = s1 + s3;
      }
    }
  }
}

template <int MU, int SGN, typename T>
__device__ inline void accumulate(Cx<T>* acc, const Cx<T> (*w)[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const Cx<T> w0 = w[0][c], w1 = w[1][c];
    acc[c] = acc[c] + w0;
    acc[3 + c] = acc[3 + c] + w1;
    if constexpr (MU == 0) {
      if constexpr (SGN < 0) {
        acc[6 + c] = acc[6 + c] + times_mi(w1);
        acc[9 + c] = acc[9 + c] + times_mi(w0);
      } else {
        acc[6 + c] = acc[6 + c] + times_i(w1);
        acc[9 + c] = acc[9 + c] + times_i(w0);
      }
    } else if constexpr (MU == 1) {
      if constexpr (SGN < 0) {
        acc[6 + c] = acc[6 + c] - w1;
        acc[9 + c] = acc[9 + c] + w0;
      } else {
        acc[6 + c] = acc[6 + c] + w1;
        acc[9 + c] = acc[9 + c] - w0;
      }
    } else if constexpr (MU == 2) {
      if constexpr (SGN < 0) {
        acc[6 + c] = acc[6 + c] + times_mi(w0);
        acc[9 + c] = acc[9 + c] + times_i(w1);
      } else {
        acc[6 + c] = acc[6 + c] + times_i(w0);
        acc[9 + c] = acc[9 + c] + times_mi(w1);
      }
    } else {
      if constexpr (SGN < 0) {
        acc[6 + c] = acc[6 + c] - w0;
        acc[9 + c] = acc[9 + c] - w1;
      } else {
        acc[6 + c] = acc[6 + c] + w0;
        acc[9 + c] = acc[9 + c] + w1;
      }
    }
  }
}

// w[s] = U h[s]  (DAG = false)  or  U^dag h[s]  (DAG = true)
template <bool DAG, typename T>
__device__ inline void colour_mul(const Cx<T> (*u)[3], const Cx<T> (*h)[3], Cx<T> (*w)[3]) {
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Cx<T> r = {T(0), T(0)};
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if constexpr (DAG)
          r = r + cmul_conj(u[b][a], h[s][b]);
        else
          r = r + u[a][b] * h[s][b];
      }
      w[s][a] = r;
    }
  }
}

template <int P, int R, int MU>
__device__ inline void hop_dir(const StencilArgs& A, const char* in, int p, int h, const int* nb,
                               Cx<typename Prec<P>::real>* acc) {
  using real = typename Prec<P>::real;
  const int q = 1 - p;
  Cx<real> s[12], hs[2][3], w[2][3], u[3][3];
  // forward: U_mu(x) (1 - gamma_mu) in(x + mu)
  SpinorIO<P>::load(in, q, nb[MU], A.g.Nh, s);
  LinkIO<P, R>::load(A.links, MU, p, h, A.g.Nh, u);
  project<MU, -1>(s, hs);
  colour_mul<false>(u, hs, w);
  accumulate<MU, -1>(acc, w);
  // backward: U_mu(x - mu)^dag (1 + gamma_mu) in(x - mu)
  SpinorIO<P>::load(in, q, nb[MU + 4], A.g.Nh, s);
  LinkIO<P, R>::load(A.links, MU, q, nb[MU + 4], A.g.Nh, u);
  project<MU, +1>(s, hs);
  colour_mul<true>(u, hs, w);
  accumulate<MU, +1>(acc, w);
}

template <int P, int R, int NV>
__global__ __launch_bounds__(256) void stencil_kernel(StencilArgs A) {
  using real = typename Prec<P>::real;
  const Geo& g = A.g;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  int p, hb;
  if (A.npar == 2) {
    p = lb & 1;
    hb = lb >> 1;
  } else {
    p = A.par0;
    hb = lb;
  }
  const int h = hb * blockDim.x + threadIdx.x;
  if (h >= g.Nh) return;
  const size_t voff = static_cast<size_t>(blockIdx.y) * A.vstride;
  const char* in = static_cast<const char*>(A.in) + voff;

  int x, y, z, t, nb[8];
  site_coords(g, p, h, x, y, z, t);
  site_neighbors(g, h, x, y, z, t, nb);

  Cx<real> acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {real(0), real(0)};
  hop_dir<P, R, 0>(A, in, p, h, nb, acc);
  hop_dir<P, R, 1>(A, in, p, h, nb, acc);
  hop_dir<P, R, 2>(A, in, p, h, nb, acc);
  hop_dir<P, R, 3>(A, in, p, h, nb, acc);

  Cx<real> s[12];
  SpinorIO<P>::load(in, p, h, g.Nh, s);
  const real a = static_cast<real>(A.a), b = static_cast<real>(A.b);
  const real sg = A.g5 ? real(-1) : real(1);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    Cx<real> r = a * s[c] + b * acc[c];
    acc[c] = (c >= 6) ? sg * r : r;
  }
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    SpinorIO<P>::load(static_cast<const char*>(A.v[j]) + voff, p, h, g.Nh, s);
    const real cj = static_cast<real>(A.cv[j]);
    const real sj = ((A.g5v >> j) & 1) ? -cj : cj;
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = acc[c] + ((c >= 6) ? sj : cj) * s[c];
  }
  SpinorIO<P>::store(static_cast<char*>(A.out) + voff, p, h, g.Nh, acc);
}

template <int P, int R>
void launch_pr(const StencilArgs& A, int nrhs, hipStream_t s) {
  constexpr int BS = 256;
  const int hblocks = (A.g.Nh + BS - 1) / BS;
  dim3 grid(hblocks * A.npar, nrhs), block(BS);
  switch (A.nv) {
    case 0: hipLaunchKernelGGL((stencil_kernel<P, R, 0>), grid, block, 0, s, A); break;
    case 1: hipLaunchKernelGGL((stencil_kernel<P, R, 1>), grid, block, 0, s, A); break;
    case 2: hipLaunchKernelGGL((stencil_kernel<P, R, 2>), grid, block, 0, s, A); break;
    case 3: hipLaunchKernelGGL((stencil_kernel<P, R, 3>), grid, block, 0, s, A); break;
    default: throw Error(OVL_E_ARG, "stencil: at most 3 extra vectors");
  }
  OVL_HIP(hipGetLastError());
}

}  // namespace

void launch_stencil(const StencilArgs& A, int prec, int recon, int nrhs, hipStream_t s) {
  OVL_REQUIRE(recon == 18 || recon == 12, OVL_E_PRECISION, "link representation missing");
  count_stencil(nrhs);
  const bool r18 = recon == 18;
  switch (prec) {
    case OVL_F64: r18 ? launch_pr<OVL_F64, 18>(A, nrhs, s) : launch_pr<OVL_F64, 12>(A, nrhs, s); break;
    case OVL_F32: r18 ? launch_pr<OVL_F32, 18>(A, nrhs, s) : launch_pr<OVL_F32, 12>(A, nrhs, s); break;
    case OVL_F16: r18 ? launch_pr<OVL_F16, 18>(A, nrhs, s) : launch_pr<OVL_F16, 12>(A, nrhs, s); break;
    case OVL_BF16: r18 ? launch_pr<OVL_BF16, 18>(A, nrhs, s) : launch_pr<OVL_BF16, 12>(A, nrhs, s); break;
    default: throw Error(OVL_E_PRECISION, "unknown precision");
  }
}

}  // namespace ovl
