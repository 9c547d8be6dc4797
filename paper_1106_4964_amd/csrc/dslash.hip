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
#include <atomic>
#include <cstdlib>
#include <tuple>

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

template <int P, int R, int MU, int KR>
__device__ inline void hop_dir(const StencilArgs& A, const char* in, int p, int h, const int* nb,
                               Cx<typename Prec<P>::real> (*acc)[12]) {
  using real = typename Prec<P>::real;
  const int q = 1 - p;
  Cx<real> s[12], hs[2][3], w[2][3], u[3][3];
  // forward: U_mu(x) (1 - gamma_mu) in(x + mu), the link shared by the KR vectors
  LinkIO<P, R>::load(A.links, MU, p, h, A.g.Nh, u);
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    SpinorIO<P>::load(in + k * A.vstride, q, nb[MU], A.g.Nh, s);
    project<MU, -1>(s, hs);
    colour_mul<false>(u, hs, w);
    accumulate<MU, -1>(acc[k], w);
  }
  // backward: U_mu(x - mu)^dag (1 + gamma_mu) in(x - mu)
  LinkIO<P, R>::load(A.links, MU, q, nb[MU + 4], A.g.Nh, u);
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    SpinorIO<P>::load(in + k * A.vstride, q, nb[MU + 4], A.g.Nh, s);
    project<MU, +1>(s, hs);
    colour_mul<true>(u, hs, w);
    accumulate<MU, +1>(acc[k], w);
  }
}

// One thread: one output site and KR consecutive vectors of the batch
// (blockIdx.y selects the group), so each link is loaded and rebuilt once
// per KR right-hand sides.
template <int P, int R, int NV, int KR>
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
  const size_t voff = static_cast<size_t>(blockIdx.y) * KR * A.vstride;
  const char* in = static_cast<const char*>(A.in) + voff;

  int x, y, z, t, nb[8];
  site_coords(g, p, h, x, y, z, t);
  site_neighbors(g, h, x, y, z, t, nb);

  Cx<real> acc[KR][12];
#pragma unroll
  for (int k = 0; k < KR; ++k)
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[k][c] = {real(0), real(0)};
  hop_dir<P, R, 0, KR>(A, in, p, h, nb, acc);
  hop_dir<P, R, 1, KR>(A, in, p, h, nb, acc);
  hop_dir<P, R, 2, KR>(A, in, p, h, nb, acc);
  hop_dir<P, R, 3, KR>(A, in, p, h, nb, acc);

  const real a = static_cast<real>(A.a), b = static_cast<real>(A.b);
  const real sg = A.g5 ? real(-1) : real(1);
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    Cx<real> s[12];
    const size_t ko = voff + k * A.vstride;
    SpinorIO<P>::load(static_cast<const char*>(A.in) + ko, p, h, g.Nh, s);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      Cx<real> r = a * s[c] + b * acc[k][c];
      acc[k][c] = (c >= 6) ? sg * r : r;
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      SpinorIO<P>::load(static_cast<const char*>(A.v[j]) + ko, p, h, g.Nh, s);
      const real cj = static_cast<real>(A.cv[j]);
      const real sj = ((A.g5v >> j) & 1) ? -cj : cj;
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[k][c] = acc[k][c] + ((c >= 6) ? sj : cj) * s[c];
    }
    SpinorIO<P>::store(static_cast<char*>(A.out) + ko, p, h, g.Nh, acc[k]);
  }
}

struct Shape {
  int kr;  // vectors per thread
  int bs;  // threads per block
};

template <int P, int R, int NV>
void launch_k(const StencilArgs& A, int nrhs, Shape sh, hipStream_t s) {
  const int hblocks = (A.g.Nh + sh.bs - 1) / sh.bs;
  dim3 grid(hblocks * A.npar, nrhs / sh.kr), block(sh.bs);
  switch (sh.kr) {
    case 1: hipLaunchKernelGGL((stencil_kernel<P, R, NV, 1>), grid, block, 0, s, A); break;
    case 2: hipLaunchKernelGGL((stencil_kernel<P, R, NV, 2>), grid, block, 0, s, A); break;
    case 3: hipLaunchKernelGGL((stencil_kernel<P, R, NV, 3>), grid, block, 0, s, A); break;
    case 4: hipLaunchKernelGGL((stencil_kernel<P, R, NV, 4>), grid, block, 0, s, A); break;
    default: throw Error(OVL_E_ARG, "stencil: unsupported vectors per thread");
  }
}

template <int P, int R>
void launch_pr(const StencilArgs& A, int nrhs, Shape sh, hipStream_t s) {
  switch (A.nv) {
    case 0: launch_k<P, R, 0>(A, nrhs, sh, s); break;
    case 1: launch_k<P, R, 1>(A, nrhs, sh, s); break;
    case 2: launch_k<P, R, 2>(A, nrhs, sh, s); break;
    case 3: launch_k<P, R, 3>(A, nrhs, sh, s); break;
    default: throw Error(OVL_E_ARG, "stencil: at most 3 extra vectors");
  }
  OVL_HIP(hipGetLastError());
}

void launch_shape(const StencilArgs& A, int prec, int recon, int nrhs, Shape sh, hipStream_t s) {
  const bool r18 = recon == 18;
  switch (prec) {
    case OVL_F64: r18 ? launch_pr<OVL_F64, 18>(A, nrhs, sh, s) : launch_pr<OVL_F64, 12>(A, nrhs, sh, s); break;
    case OVL_F32: r18 ? launch_pr<OVL_F32, 18>(A, nrhs, sh, s) : launch_pr<OVL_F32, 12>(A, nrhs, sh, s); break;
    case OVL_F16: r18 ? launch_pr<OVL_F16, 18>(A, nrhs, sh, s) : launch_pr<OVL_F16, 12>(A, nrhs, sh, s); break;
    case OVL_BF16: r18 ? launch_pr<OVL_BF16, 18>(A, nrhs, sh, s) : launch_pr<OVL_BF16, 12>(A, nrhs, sh, s); break;
    default: throw Error(OVL_E_PRECISION, "unknown precision");
  }
}

// ------------------------------------------------------------------ tuner
// The shape (vectors per thread, block size) of each stencil configuration
// is chosen once per process by timing every candidate with HIP events on a
// scratch output; OVL_TUNE=0 keeps the static default.  Results are cached
// in memory, keyed by precision, link format, extra vectors, batch size,
// output parities and lattice volume.
struct TuneKey {
  int prec, recon, nv, nrhs, npar, nh;
  bool operator<(const TuneKey& o) const {
    return std::tie(prec, recon, nv, nrhs, npar, nh) < std::tie(o.prec, o.recon, o.nv, o.nrhs, o.npar, o.nh);
  }
};

std::mutex g_tune_mu;
std::map<TuneKey, Shape> g_tuned;

std::atomic<int> g_tune_mode{-1};  // -1: not read yet, 0: static default, 1: autotune

bool tuning_enabled() {
  int m = g_tune_mode.load();
  if (m < 0) {
    const char* e = std::getenv("OVL_TUNE");
    m = (e && e[0] == '0') ? 0 : 1;
    g_tune_mode.store(m);
  }
  return m == 1;
}

std::vector<Shape> candidates(int prec, int nrhs) {
  std::vector<Shape> c;
  const int kmax = prec == OVL_F64 ? 2 : 4;
  for (int kr = 1; kr <= kmax; ++kr)
    if (nrhs % kr == 0)
      for (int bs : {128, 256}) c.push_back({kr, bs});
  return c;
}

Shape default_shape(int prec, int nrhs) {
  const int kmax = prec == OVL_F64 ? 2 : 4;
  for (int kr = kmax; kr >= 1; --kr)
    if (nrhs % kr == 0) return {kr, 256};
  return {1, 256};
}

Shape pick_shape(const StencilArgs& A, int prec, int recon, int nrhs, hipStream_t s) {
  const TuneKey key{prec, recon, A.nv, nrhs, A.npar, A.g.Nh};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second;
  }
  const Shape def = default_shape(prec, nrhs);
  if (!tuning_enabled()) return def;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return def;
  // time every candidate on a scratch output (the real output may alias an input)
  StencilArgs T = A;
  WsBuf scratch(A.vstride * nrhs, s);
  T.out = scratch.p;
  hipEvent_t e0, e1;
  OVL_HIP(hipEventCreate(&e0));
  OVL_HIP(hipEventCreate(&e1));
  Shape best = def;
  float best_ms = 1e30f;
  for (const Shape& c : candidates(prec, nrhs)) {
    launch_shape(T, prec, recon, nrhs, c, s);  // warm-up
    OVL_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < 3; ++r) launch_shape(T, prec, recon, nrhs, c, s);
    OVL_HIP(hipEventRecord(e1, s));
    OVL_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    OVL_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  OVL_HIP(hipEventDestroy(e0));
  OVL_HIP(hipEventDestroy(e1));
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = best;
  return best;
}

}  // namespace

void launch_stencil(const StencilArgs& A, int prec, int recon, int nrhs, hipStream_t s) {
  OVL_REQUIRE(recon == 18 || recon == 12, OVL_E_PRECISION, "link representation missing");
  count_stencil(nrhs);
  const Shape sh = pick_shape(A, prec, recon, nrhs, s);
  launch_shape(A, prec, recon, nrhs, sh, s);
}

void set_tune_mode(int mode) {
  g_tune_mode.store(mode ? 1 : 0);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned.clear();
}

int stencil_shape(int prec, int recon, int nv, int nrhs, int npar, int nh, int* kr, int* bs) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(TuneKey{prec, recon, nv, nrhs, npar, nh});
  if (it == g_tuned.end()) return 0;
  *kr = it->second.kr;
  *bs = it->second.bs;
  return 1;
}

}  // namespace ovl
