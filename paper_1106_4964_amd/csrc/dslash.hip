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
#include <algorithm>
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
// h_k = s_k + phase * s_partner with phase +1, -1, +i, -i coded 0, 1, 2, 3
// (code ^ 1 negates).
template <int PH, typename T>
__device__ inline Cx<T> proj1(Cx<T> a, Cx<T> b) {
  if constexpr (PH == 0) return {a.re + b.re, a.im + b.im};
  else if constexpr (PH == 1) return {a.re - b.re, a.im - b.im};
  else if constexpr (PH == 2) return {a.re - b.im, a.im + b.re};  // + i b
  else return {a.re + b.im, a.im - b.re};                          // - i b
}

template <int MU, int SGN, typename T>
__device__ inline void project(const Cx<T>* s, Cx<T> (*h)[3]) {
  constexpr int p0 = MU < 2 ? 3 : 2, p1 = MU < 2 ? 2 : 3;
  constexpr int f = SGN < 0 ? 0 : 1;
  constexpr int ph0 = (MU == 0 ? 2 : MU == 1 ? 0 : MU == 2 ? 2 : 1) ^ f;
  constexpr int ph1 = (MU == 0 ? 2 : MU == 1 ? 1 : MU == 2 ? 3 : 1) ^ f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    h[0][c] = proj1<ph0>(s[c], s[3 * p0 + c]);
    h[1][c] = proj1<ph1>(s[3 + c], s[3 * p1 + c]);
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

// re + i im += u h  (CONJ: conj(u) h), four FMAs.
template <bool CONJ, typename T>
__device__ inline void cmac(T& re, T& im, Cx<T> u, Cx<T> h) {
  re = ffma(u.re, h.re, re);
  im = ffma(u.re, h.im, im);
  if constexpr (CONJ) {
    re = ffma(u.im, h.im, re);
    im = ffma(-u.im, h.re, im);
  } else {
    re = ffma(-u.im, h.im, re);
    im = ffma(u.im, h.re, im);
  }
}

// sum_b u_b h_b (CONJ: conj(u_b) h_b).  CHAIN: one FMA chain per real part
// (4 instructions per complex multiply-add); otherwise products summed as a
// tree (6 instructions, shorter dependence chains, fewer live registers).
// Which is faster depends on the format (measured): chains for FP64, FP32
// and BF16, the tree for F16.
template <bool CONJ, bool CHAIN, typename T>
__device__ inline Cx<T> row3(Cx<T> u0, Cx<T> u1, Cx<T> u2, const Cx<T>* h) {
  if constexpr (CHAIN) {
    T re = T(0), im = T(0);
    cmac<CONJ>(re, im, u0, h[0]);
    cmac<CONJ>(re, im, u1, h[1]);
    cmac<CONJ>(re, im, u2, h[2]);
    return {re, im};
  } else if constexpr (CONJ) {
    return cmul_conj(u0, h[0]) + cmul_conj(u1, h[1]) + cmul_conj(u2, h[2]);
  } else {
    return u0 * h[0] + u1 * h[1] + u2 * h[2];
  }
}

// w[s] = U h[s]  (DAG = false)  or  U^dag h[s]  (DAG = true)
template <bool DAG, bool CHAIN, typename T>
__device__ inline void colour_mul(const Cx<T> (*u)[3], const Cx<T> (*h)[3], Cx<T> (*w)[3]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a)
      w[s][a] = DAG ? row3<true, CHAIN>(u[0][a], u[1][a], u[2][a], h[s])
                    : row3<false, CHAIN>(u[a][0], u[a][1], u[a][2], h[s]);
}

// FMA chains (fewer instructions) everywhere except the FP16 kernels with
// extra epilogue vectors, where the pairwise-summed form measured faster.
// FP16 chains take their operands through opaque(): otherwise the compiler
// folds the FP16->FP32 conversions into mixed-precision FMAs that keep the
// FP16 inputs live across the chains (about 200 VGPRs).
template <int P, int NV>
constexpr bool chain_form() {
  return P != OVL_F16 || NV == 0;
}

template <int P, bool CH, int N>
__device__ inline void opaque(Cx<float>* v) {
  if constexpr (P == OVL_F16 && CH) {
#pragma unroll
    for (int i = 0; i < N; ++i) asm("" : "+v"(v[i].re), "+v"(v[i].im));
  }
}
template <int P, bool CH, int N>
__device__ inline void opaque(Cx<double>*) {}

template <int P, int R, int MU, int KR, bool CH>
__device__ inline void hop_dir(const StencilArgs& A, const char* in, int p, int h, const int* nb,
                               Cx<typename Prec<P>::real> (*acc)[12]) {
  using real = typename Prec<P>::real;
  const int q = 1 - p;
  Cx<real> s[12], hs[2][3], w[2][3], u[3][3];
  // forward: U_mu(x) (1 - gamma_mu) in(x + mu), the link shared by the KR vectors
  LinkIO<P, R>::load(A.links, MU, p, h, A.g.Nh, u);
  opaque<P, CH, 9>(&u[0][0]);
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    SpinorIO<P>::load(in + k * A.vstride, q, nb[MU], A.g.Nh, s);
    opaque<P, CH, 12>(s);
    project<MU, -1>(s, hs);
    colour_mul<false, CH>(u, hs, w);
    accumulate<MU, -1>(acc[k], w);
  }
  // backward: U_mu(x - mu)^dag (1 + gamma_mu) in(x - mu)
  LinkIO<P, R>::load(A.links, MU, q, nb[MU + 4], A.g.Nh, u);
  opaque<P, CH, 9>(&u[0][0]);
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    SpinorIO<P>::load(in + k * A.vstride, q, nb[MU + 4], A.g.Nh, s);
    opaque<P, CH, 12>(s);
    project<MU, +1>(s, hs);
    colour_mul<true, CH>(u, hs, w);
    accumulate<MU, +1>(acc[k], w);
  }
}

// Epilogue at the output site: G(a*in + b*hop) + sum_j c_j G_j(v_j), G = 1
// or gamma5, then the store.
template <int P, int NV>
__device__ inline void epilogue(const StencilArgs& A, size_t off, int p, int h, Cx<typename Prec<P>::real>* acc) {
  using real = typename Prec<P>::real;
  const real a = static_cast<real>(A.a), b = static_cast<real>(A.b);
  const real sg = A.g5 ? real(-1) : real(1);
  Cx<real> s[12];
  SpinorIO<P>::load(static_cast<const char*>(A.in) + off, p, h, A.g.Nh, s);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const Cx<real> r = a * s[c] + b * acc[c];
    acc[c] = (c >= 6) ? sg * r : r;
  }
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    SpinorIO<P>::load_nt(static_cast<const char*>(A.v[j]) + off, p, h, A.g.Nh, s);
    const real cj = static_cast<real>(A.cv[j]);
    const real sj = ((A.g5v >> j) & 1) ? -cj : cj;
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = acc[c] + ((c >= 6) ? sj : cj) * s[c];
  }
  SpinorIO<P>::store_nt(static_cast<char*>(A.out) + off, p, h, A.g.Nh, acc);
}

// Output site (parity p, half index h) of this thread; false past the end.
__device__ inline bool stencil_site(const StencilArgs& A, int& p, int& h) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  int hb;
  if (A.npar == 2) {
    p = lb & 1;
    hb = lb >> 1;
  } else {
    p = A.par0;
    hb = lb;
  }
  if (A.tmaj) {
    const int tile = hb / A.g.Lt, t = hb - tile * A.g.Lt;
    const int hl = tile * blockDim.x + threadIdx.x;
    h = t * A.g.st + hl;
    return hl < A.g.st;
  }
  h = hb * blockDim.x + threadIdx.x;
  return h < A.g.Nh;
}

// One thread: one output site and KR consecutive vectors of the batch, so
// each link is loaded and rebuilt once per KR right-hand sides.  With
// RIN = false the group of KR vectors is blockIdx.y (one pass over the
// lattice per group); with RIN = true it is threadIdx.y, so all groups of a
// site tile run in the same workgroup and share its links and neighbour
// spinors through L1/L2 (one pass over the lattice for the whole batch).
template <int P, int R, int NV, int KR, bool RIN>
__global__ __launch_bounds__(RIN ? 512 : 256) void stencil_kernel(StencilArgs A) {
  using real = typename Prec<P>::real;
  const Geo& g = A.g;
  int p, h;
  if (!stencil_site(A, p, h)) return;
  const int group = RIN ? threadIdx.y : blockIdx.y;
  const size_t voff = static_cast<size_t>(group) * KR * A.vstride;
  const char* in = static_cast<const char*>(A.in) + voff;

  int x, y, z, t, nb[8];
  site_coords(g, p, h, x, y, z, t);
  site_neighbors(g, h, x, y, z, t, nb);

  Cx<real> acc[KR][12];
#pragma unroll
  for (int k = 0; k < KR; ++k)
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[k][c] = {real(0), real(0)};
  hop_dir<P, R, 0, KR, chain_form<P, NV>()>(A, in, p, h, nb, acc);
  hop_dir<P, R, 1, KR, chain_form<P, NV>()>(A, in, p, h, nb, acc);
  hop_dir<P, R, 2, KR, chain_form<P, NV>()>(A, in, p, h, nb, acc);
  hop_dir<P, R, 3, KR, chain_form<P, NV>()>(A, in, p, h, nb, acc);

#pragma unroll
  for (int k = 0; k < KR; ++k) epilogue<P, NV>(A, voff + k * A.vstride, p, h, acc[k]);
}

// Software-pipelined variant for one vector per thread: the raw loads of
// direction D + DEP - 1 are issued before the arithmetic of direction D, so
// DEP directions' worth of loads are in flight per wave.  Directions run
// +x, -x, +y, -y, ... (D = 2 mu + backward).
template <int P, int R, int D>
__device__ inline void pipe_issue(const StencilArgs& A, const char* in, int p, int h, const int* nb,
                                  SpinorRaw<P>& sr, LinkRaw<P, R>& lr) {
  constexpr int MU = D / 2;
  const int q = 1 - p;
  if constexpr (D % 2 == 0) {
    spinor_load_raw<P>(in, q, nb[MU], A.g.Nh, sr);
    link_load_raw<P, R>(A.links, MU, p, h, A.g.Nh, lr);
  } else {
    spinor_load_raw<P>(in, q, nb[MU + 4], A.g.Nh, sr);
    link_load_raw<P, R>(A.links, MU, q, nb[MU + 4], A.g.Nh, lr);
  }
}

template <int P, int R, int D>
__device__ inline void pipe_consume(const SpinorRaw<P>& sr, const LinkRaw<P, R>& lr,
                                    Cx<typename Prec<P>::real>* acc) {
  using real = typename Prec<P>::real;
  constexpr int MU = D / 2;
  constexpr bool CH = P != OVL_F16;  // the pipelined kernels keep the pairwise form for FP16
  Cx<real> s[12], hs[2][3], w[2][3], u[3][3];
  spinor_unpack<P>(sr, s);
  link_unpack<P, R>(lr, u);
  if constexpr (D % 2 == 0) {
    project<MU, -1>(s, hs);
    colour_mul<false, CH>(u, hs, w);
    accumulate<MU, -1>(acc, w);
  } else {
    project<MU, +1>(s, hs);
    colour_mul<true, CH>(u, hs, w);
    accumulate<MU, +1>(acc, w);
  }
}

template <int P, int R, int DEP, int D>
__device__ inline void pipe_run(const StencilArgs& A, const char* in, int p, int h, const int* nb,
                                SpinorRaw<P> (&sr)[DEP], LinkRaw<P, R> (&lr)[DEP],
                                Cx<typename Prec<P>::real>* acc) {
  if constexpr (D + DEP - 1 < 8) pipe_issue<P, R, D + DEP - 1>(A, in, p, h, nb, sr[(D + DEP - 1) % DEP], lr[(D + DEP - 1) % DEP]);
  pipe_consume<P, R, D>(sr[D % DEP], lr[D % DEP], acc);
  if constexpr (D + 1 < 8) pipe_run<P, R, DEP, D + 1>(A, in, p, h, nb, sr, lr, acc);
}

template <int P, int R, int DEP, int D>
__device__ inline void pipe_prologue(const StencilArgs& A, const char* in, int p, int h, const int* nb,
                                     SpinorRaw<P> (&sr)[DEP], LinkRaw<P, R> (&lr)[DEP]) {
  if constexpr (D < DEP - 1) {
    pipe_issue<P, R, D>(A, in, p, h, nb, sr[D], lr[D]);
    pipe_prologue<P, R, DEP, D + 1>(A, in, p, h, nb, sr, lr);
  }
}

template <int P, int R, int NV, int DEP>
__global__ __launch_bounds__(256) void stencil_pipe_kernel(StencilArgs A) {
  using real = typename Prec<P>::real;
  const Geo& g = A.g;
  int p, h;
  if (!stencil_site(A, p, h)) return;
  const size_t voff = static_cast<size_t>(blockIdx.y) * A.vstride;
  const char* in = static_cast<const char*>(A.in) + voff;
  int x, y, z, t, nb[8];
  site_coords(g, p, h, x, y, z, t);
  site_neighbors(g, h, x, y, z, t, nb);
  SpinorRaw<P> sr[DEP];
  LinkRaw<P, R> lr[DEP];
  pipe_prologue<P, R, DEP, 0>(A, in, p, h, nb, sr, lr);
  Cx<real> acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {real(0), real(0)};
  pipe_run<P, R, DEP, 0>(A, in, p, h, nb, sr, lr, acc);
  epilogue<P, NV>(A, voff, p, h, acc);
}

struct Shape {
  int kr;    // vectors per thread
  int bs;    // threads per block (sites per block when rin)
  int pipe;  // 0: plain kernel; >= 2: pipelined one-vector kernel of that depth
  int rin;   // 1: the nrhs/kr vector groups are the y-dimension of the block
  int tm;    // 1: t-major block order (StencilArgs::tmaj)
};

template <int P, int R, int NV>
void launch_k(const StencilArgs& A0, int nrhs, Shape sh, hipStream_t s) {
  StencilArgs A = A0;
  A.tmaj = sh.tm;
  const int hblocks = sh.tm ? ((A.g.st + sh.bs - 1) / sh.bs) * A.g.Lt : (A.g.Nh + sh.bs - 1) / sh.bs;
  if (sh.rin) {
    const int groups = nrhs / sh.kr;
    OVL_REQUIRE(sh.bs * groups <= 512, OVL_E_ARG, "stencil: block too large");
    dim3 grid(hblocks * A.npar), block(sh.bs, groups);
    switch (sh.kr) {
      case 1: hipLaunchKernelGGL((stencil_kernel<P, R, NV, 1, true>), grid, block, 0, s, A); break;
      case 2: hipLaunchKernelGGL((stencil_kernel<P, R, NV, 2, true>), grid, block, 0, s, A); break;
      case 3: hipLaunchKernelGGL((stencil_kernel<P, R, NV, 3, true>), grid, block, 0, s, A); break;
      case 4: hipLaunchKernelGGL((stencil_kernel<P, R, NV, 4, true>), grid, block, 0, s, A); break;
      default: throw Error(OVL_E_ARG, "stencil: unsupported vectors per thread");
    }
    return;
  }
  dim3 grid(hblocks * A.npar, nrhs / sh.kr), block(sh.bs);
  if (sh.pipe) {
    switch (sh.pipe) {
      case 2: hipLaunchKernelGGL((stencil_pipe_kernel<P, R, NV, 2>), grid, block, 0, s, A); break;
      case 3: hipLaunchKernelGGL((stencil_pipe_kernel<P, R, NV, 3>), grid, block, 0, s, A); break;
      case 4: hipLaunchKernelGGL((stencil_pipe_kernel<P, R, NV, 4>), grid, block, 0, s, A); break;
      default: throw Error(OVL_E_ARG, "stencil: unsupported pipeline depth");
    }
    return;
  }
  switch (sh.kr) {
    case 1: hipLaunchKernelGGL((stencil_kernel<P, R, NV, 1, false>), grid, block, 0, s, A); break;
    case 2: hipLaunchKernelGGL((stencil_kernel<P, R, NV, 2, false>), grid, block, 0, s, A); break;
    case 3: hipLaunchKernelGGL((stencil_kernel<P, R, NV, 3, false>), grid, block, 0, s, A); break;
    case 4: hipLaunchKernelGGL((stencil_kernel<P, R, NV, 4, false>), grid, block, 0, s, A); break;
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
  for (int tm = 0; tm <= 1; ++tm) {
    for (int kr = 1; kr <= kmax; ++kr)
      if (nrhs % kr == 0) {
        for (int bs : {128, 256}) c.push_back({kr, bs, 0, 0, tm});
        if (nrhs > kr)  // several groups: try them side by side in one workgroup
          for (int bs : {32, 64})
            if (bs * (nrhs / kr) <= 512) c.push_back({kr, bs, 0, 1, tm});
      }
    for (int dep : {2, 3, 4})
      if (prec != OVL_F64 || dep == 2)
        for (int bs : {128, 256}) c.push_back({1, bs, dep, 0, tm});
  }
  return c;
}

Shape default_shape(int prec, int nrhs) {
  const int kmax = prec == OVL_F64 ? 2 : 4;
  for (int kr = kmax; kr >= 1; --kr)
    if (nrhs % kr == 0) return {kr, 256, 0, 0, 0};
  return {1, 256, 0, 0, 0};
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
  // two rounds over the candidates, each timed over 3 launches after a
  // warm-up launch; a candidate's time is its better round.  The first
  // candidate (in list order) within 2% of the fastest wins, so that shapes
  // that time alike give the same choice from run to run.
  const std::vector<Shape> cand = candidates(prec, nrhs);
  std::vector<float> best_ms(cand.size(), 1e30f);
  for (int round = 0; round < 2; ++round)
    for (size_t i = 0; i < cand.size(); ++i) {
      launch_shape(T, prec, recon, nrhs, cand[i], s);  // warm-up
      OVL_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 3; ++r) launch_shape(T, prec, recon, nrhs, cand[i], s);
      OVL_HIP(hipEventRecord(e1, s));
      OVL_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      OVL_HIP(hipEventElapsedTime(&ms, e0, e1));
      best_ms[i] = std::min(best_ms[i], ms);
    }
  float fastest = 1e30f;
  for (float t : best_ms) fastest = std::min(fastest, t);
  Shape best = def;
  for (size_t i = 0; i < cand.size(); ++i)
    if (best_ms[i] <= 1.02f * fastest) {
      best = cand[i];
      break;
    }
  OVL_HIP(hipEventDestroy(e0));
  OVL_HIP(hipEventDestroy(e1));
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = best;
  return best;
}

}  // namespace

// Per-configuration launch timer: HIP events recorded on the launch stream
// around each stencil launch while enabled (not during stream capture).
namespace {
struct TimerKey {
  int prec, recon, nv, nrhs;
  bool operator<(const TimerKey& o) const {
    return std::tie(prec, recon, nv, nrhs) < std::tie(o.prec, o.recon, o.nv, o.nrhs);
  }
};
struct TimerRec {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  int64_t launches = 0;
  double ms = 0.0;
};
std::atomic<bool> g_timing{false};
std::mutex g_timer_mu;
std::map<TimerKey, TimerRec> g_timer;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t timer_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  OVL_HIP(hipEventCreate(&e));
  return e;
}

void timer_settle(TimerRec& r) {
  for (auto& pr : r.pending) {
    OVL_HIP(hipEventSynchronize(pr.second));
    float ms = 0.f;
    OVL_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
    r.ms += ms;
    r.launches += 1;
    g_event_pool.push_back(pr.first);
    g_event_pool.push_back(pr.second);
  }
  r.pending.clear();
}
}  // namespace

void launch_stencil(const StencilArgs& A, int prec, int recon, int nrhs, hipStream_t s) {
  OVL_REQUIRE(recon == 18 || recon == 12, OVL_E_PRECISION, "link representation missing");
  count_stencil(nrhs);
  const Shape sh = pick_shape(A, prec, recon, nrhs, s);
  bool timed = false;
  if (g_timing.load(std::memory_order_relaxed)) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    timed = hipStreamIsCapturing(s, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone;
  }
  if (!timed) {
    launch_shape(A, prec, recon, nrhs, sh, s);
    return;
  }
  std::lock_guard<std::mutex> lk(g_timer_mu);
  hipEvent_t e0 = timer_event(), e1 = timer_event();
  OVL_HIP(hipEventRecord(e0, s));
  launch_shape(A, prec, recon, nrhs, sh, s);
  OVL_HIP(hipEventRecord(e1, s));
  g_timer[TimerKey{prec, recon, A.nv, nrhs}].pending.emplace_back(e0, e1);
}

void stencil_timer(int mode) {
  std::lock_guard<std::mutex> lk(g_timer_mu);
  if (mode == 1 || mode == 2) {
    for (auto& kv : g_timer) timer_settle(kv.second);
    g_timer.clear();
  }
  if (mode == 0 || mode == 1) g_timing.store(mode == 1);
}

void stencil_timer_read(int prec, int recon, int nv, int nrhs, int64_t* launches, double* ms) {
  std::lock_guard<std::mutex> lk(g_timer_mu);
  auto it = g_timer.find(TimerKey{prec, recon, nv, nrhs});
  if (it == g_timer.end()) {
    *launches = 0;
    *ms = 0.0;
    return;
  }
  timer_settle(it->second);
  *launches = it->second.launches;
  *ms = it->second.ms;
}

void set_tune_mode(int mode) {
  g_tune_mode.store(mode ? 1 : 0);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned.clear();
}

int stencil_shape(int prec, int recon, int nv, int nrhs, int npar, int nh, int* shape5) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(TuneKey{prec, recon, nv, nrhs, npar, nh});
  if (it == g_tuned.end()) return 0;
  const Shape& sh = it->second;
  shape5[0] = sh.kr;
  shape5[1] = sh.bs;
  shape5[2] = sh.pipe;
  shape5[3] = sh.rin;
  shape5[4] = sh.tm;
  return 1;
}

void force_shape(int prec, int recon, int nv, int nrhs, int npar, int nh, const int* shape5) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[TuneKey{prec, recon, nv, nrhs, npar, nh}] = Shape{shape5[0], shape5[1], shape5[2], shape5[3], shape5[4]};
}

}  // namespace ovl
