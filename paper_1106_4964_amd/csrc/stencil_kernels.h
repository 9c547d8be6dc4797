// Wilson hopping stencil kernels (arXiv:1106.4964 Sec. II, eq. 1-2) with
// fused epilogues: the device templates and their launchers.  Each storage
// precision and link format is instantiated in a translation unit of its own
// (stencil_<prec>.hip), so the kernels compile in parallel.
//
// One thread computes the 12 complex output components of one site for KR
// right-hand sides.  For each of the 8 directions it loads the neighbour
// spinor, spin-projects it to a 2x3 half spinor with (1 -+ gamma_mu),
// multiplies both colour vectors by U_mu(x) or U_mu(x-mu)^dag and adds the
// result back, the lower two spin components being fixed multiples of the
// upper two (chiral basis).  The epilogue forms
// G(a*in + b*hop) + sum_j c_j G_j(v_j) at the output site, which covers
// D_w(m), H_w = gamma5 D_w(-rho), and the Clenshaw update of the polynomial
// sign function (Sec. V) in one pass.
#pragma once

#include "ops.h"

namespace ovl {

struct Shape {
  int kr;    // vectors per thread
  int bs;    // threads per block (sites per block when rin)
  int pipe;  // 0: plain kernel; >= 2: pipelined one-vector kernel of that depth
  int rin;   // 1: the nrhs/kr vector groups are the y-dimension of the block
  int tm;    // block order (StencilArgs::tmaj): 0 by h, 1 t-major, >= 2 z-slabs of tm planes
};

// Launches the stencil in shape sh for one storage precision (one function
// per translation unit).
void launch_stencil_f64(const StencilArgs& A, int recon, int nrhs, Shape sh, hipStream_t s);
void launch_stencil_f32(const StencilArgs& A, int recon, int nrhs, Shape sh, hipStream_t s);
void launch_stencil_f16(const StencilArgs& A, int recon, int nrhs, Shape sh, hipStream_t s);
void launch_stencil_bf16(const StencilArgs& A, int recon, int nrhs, Shape sh, hipStream_t s);

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

// acc += s * ph * w for the phase ph coded as in proj1 (0: +1, 1: -1, 2: +i,
// 3: -i), two FMAs (the sign of s is a source modifier).
template <int PH, typename T>
__device__ inline void addph(Cx<T>& a, Cx<T> w, T s) {
  if constexpr (PH == 0) {
    a.re = ffma(s, w.re, a.re);
    a.im = ffma(s, w.im, a.im);
  } else if constexpr (PH == 1) {
    a.re = ffma(-s, w.re, a.re);
    a.im = ffma(-s, w.im, a.im);
  } else if constexpr (PH == 2) {  // + i w = (-w.im, w.re)
    a.re = ffma(-s, w.im, a.re);
    a.im = ffma(s, w.re, a.im);
  } else {  // - i w = (w.im, -w.re)
    a.re = ffma(s, w.im, a.re);
    a.im = ffma(-s, w.re, a.im);
  }
}

// Adds the reconstructed direction term: upper spins += bu * w, lower spins
// += bl * (phase) w.  bu = b and bl = +-b carry the hopping weight of the
// epilogue and, for gamma5 outputs, the sign of the lower spins, so neither
// costs an instruction of its own.
template <int MU, int SGN, typename T>
__device__ inline void accumulate(Cx<T>* acc, const Cx<T> (*w)[3], T bu, T bl) {
  // phase code and source spin (0 or 1) of lower spins 2 and 3
  constexpr bool F = SGN < 0;
  constexpr int l0 = MU == 0 ? (F ? 3 : 2) : MU == 1 ? (F ? 1 : 0) : MU == 2 ? (F ? 3 : 2) : (F ? 1 : 0);
  constexpr int l1 = MU == 0 ? (F ? 3 : 2) : MU == 1 ? (F ? 0 : 1) : MU == 2 ? (F ? 2 : 3) : (F ? 1 : 0);
  constexpr int s0 = MU < 2 ? 1 : 0, s1 = MU < 2 ? 0 : 1;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    addph<0>(acc[c], w[0][c], bu);
    addph<0>(acc[3 + c], w[1][c], bu);
    addph<l0>(acc[6 + c], w[s0][c], bl);
    addph<l1>(acc[9 + c], w[s1][c], bl);
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

// ------------------------------------------------------- F16 operands
// An F16 spinor is 12 dwords, dword c holding complex component
// c = 3*spin + colour as (re, im) halves.  v_fma_mix_f32 takes an f16 half of
// a dword as an operand and computes in f32, so the spin projection and the
// epilogue read the stored halves directly: one instruction per real
// instead of a conversion plus the arithmetic.
//   mix_pm<HB, HA, NEG>(b, a) = (NEG ? -1 : +1) * half(b, HB) + half(a, HA)
//   mix_fma<HA>(a, s, c)      = half(a, HA) * s + c
// (half 0 = low, 1 = high; s and c in f32; s uniform, in an SGPR).
#define OVL_MIX_PM(HB, HA, K)                                                                             \
  asm("v_fma_mix_f32 %0, %1, " K ", %2 op_sel:[" #HB ",0," #HA "] op_sel_hi:[1,0,1]" : "=v"(d) : "v"(b), \
      "v"(a))
template <int HB, int HA, bool NEG>
__device__ inline float mix_pm(uint32_t b, uint32_t a) {
  float d;
  if constexpr (HB == 0 && HA == 0) {
    if constexpr (NEG) OVL_MIX_PM(0, 0, "-1.0"); else OVL_MIX_PM(0, 0, "1.0");
  } else if constexpr (HB == 0 && HA == 1) {
    if constexpr (NEG) OVL_MIX_PM(0, 1, "-1.0"); else OVL_MIX_PM(0, 1, "1.0");
  } else if constexpr (HB == 1 && HA == 0) {
    if constexpr (NEG) OVL_MIX_PM(1, 0, "-1.0"); else OVL_MIX_PM(1, 0, "1.0");
  } else {
    if constexpr (NEG) OVL_MIX_PM(1, 1, "-1.0"); else OVL_MIX_PM(1, 1, "1.0");
  }
  return d;
}
#undef OVL_MIX_PM

template <int HA>
__device__ inline float mix_fma(uint32_t a, float s, float c) {
  float d;
  if constexpr (HA == 0)
    asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[0,0,0] op_sel_hi:[1,0,0]" : "=v"(d) : "v"(a), "s"(s), "v"(c));
  else
    asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(d) : "v"(a), "s"(s), "v"(c));
  return d;
}

// a + ph * b for complex components given as (re, im) f16 dwords
template <int PH>
__device__ inline Cx<float> proj1_f16(uint32_t a, uint32_t b) {
  if constexpr (PH == 0) return {mix_pm<0, 0, false>(b, a), mix_pm<1, 1, false>(b, a)};
  else if constexpr (PH == 1) return {mix_pm<0, 0, true>(b, a), mix_pm<1, 1, true>(b, a)};
  else if constexpr (PH == 2) return {mix_pm<1, 0, true>(b, a), mix_pm<0, 1, false>(b, a)};  // + i b
  else return {mix_pm<1, 0, false>(b, a), mix_pm<0, 1, true>(b, a)};                          // - i b
}

// (1 + SGN gamma_mu) psi -> h[2][3] straight from the raw F16 dwords
template <int MU, int SGN>
__device__ inline void project_f16(const uint32_t* s, Cx<float> (*h)[3]) {
  constexpr int p0 = MU < 2 ? 3 : 2, p1 = MU < 2 ? 2 : 3;
  constexpr int f = SGN < 0 ? 0 : 1;
  constexpr int ph0 = (MU == 0 ? 2 : MU == 1 ? 0 : MU == 2 ? 2 : 1) ^ f;
  constexpr int ph1 = (MU == 0 ? 2 : MU == 1 ? 1 : MU == 2 ? 3 : 1) ^ f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    h[0][c] = proj1_f16<ph0>(s[c], s[3 * p0 + c]);
    h[1][c] = proj1_f16<ph1>(s[3 + c], s[3 * p1 + c]);
  }
}

__device__ inline uint32_t raw_word(const SpinorRaw<OVL_F16>& r, int c) {
  const uint4 v = r.b[c / 4];
  const int k = c % 4;
  return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w;
}

// One FMA chain per real part of each colour row.
template <int P, int NV>
constexpr bool chain_form() {
  return true;
}

// F16 links are converted to f32 once per thread and then hidden from the
// optimiser: otherwise it folds the conversions into the colour products as
// v_fma_mix_f32, which issues at about 70% of the rate of v_fma_f32
// (measured on MI355X: 35 vs 51 T lane-instructions/s) and would run 72 of
// them per direction and vector instead of 12 conversions per link.
template <int P>
__device__ inline void opaque_link(Cx<typename Prec<P>::real> (*u)[3]) {
  if constexpr (P == OVL_F16) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) asm("" : "+v"(u[i][j].re), "+v"(u[i][j].im));
  }
}

template <int P, int R, int MU, int KR, bool CH>
__device__ inline void hop_dir(const StencilArgs& A, const char* in, int p, int h, const int* nb,
                               Cx<typename Prec<P>::real> (*acc)[12], typename Prec<P>::real bu,
                               typename Prec<P>::real bl) {
  using real = typename Prec<P>::real;
  const int q = 1 - p;
  Cx<real> hs[2][3], w[2][3], u[3][3];
  // forward: U_mu(x) (1 - gamma_mu) in(x + mu), the link shared by the KR vectors
  LinkIO<P, R>::load(A.links, MU, p, h, A.g.Nh, u);
  opaque_link<P>(u);
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    if constexpr (P == OVL_F16) {
      SpinorRaw<P> r;
      spinor_load_raw<P>(in + k * A.vstride, q, nb[MU], A.g.Nh, r);
      uint32_t sw[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) sw[c] = raw_word(r, c);
      project_f16<MU, -1>(sw, hs);
    } else {
      Cx<real> s[12];
      SpinorIO<P>::load(in + k * A.vstride, q, nb[MU], A.g.Nh, s);
      project<MU, -1>(s, hs);
    }
    colour_mul<false, CH>(u, hs, w);
    accumulate<MU, -1>(acc[k], w, bu, bl);
  }
  // backward: U_mu(x - mu)^dag (1 + gamma_mu) in(x - mu)
  LinkIO<P, R>::load(A.links, MU, q, nb[MU + 4], A.g.Nh, u);
  opaque_link<P>(u);
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    if constexpr (P == OVL_F16) {
      SpinorRaw<P> r;
      spinor_load_raw<P>(in + k * A.vstride, q, nb[MU + 4], A.g.Nh, r);
      uint32_t sw[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) sw[c] = raw_word(r, c);
      project_f16<MU, +1>(sw, hs);
    } else {
      Cx<real> s[12];
      SpinorIO<P>::load(in + k * A.vstride, q, nb[MU + 4], A.g.Nh, s);
      project<MU, +1>(s, hs);
    }
    colour_mul<true, CH>(u, hs, w);
    accumulate<MU, +1>(acc[k], w, bu, bl);
  }
}

// Hopping weights of the accumulation: b on the upper spins, and on the
// lower spins b, or -b when the output takes gamma5.
template <typename T>
__device__ inline void hop_weights(const StencilArgs& A, T& bu, T& bl) {
  bu = static_cast<T>(A.b);
  bl = A.g5 ? -bu : bu;
}

// Epilogue at the output site: G(a*in + b*hop) + sum_j c_j G_j(v_j), G = 1
// or gamma5, then the store.  acc already holds b*hop with G's sign on the
// lower spins.
template <int P, int NV>
__device__ inline void epilogue(const StencilArgs& A, size_t off, int p, int h, Cx<typename Prec<P>::real>* acc) {
  using real = typename Prec<P>::real;
  const real au = static_cast<real>(A.a), al = A.g5 ? -au : au;
  if constexpr (P == OVL_F16) {
    SpinorRaw<P> r;
    spinor_load_raw<P>(static_cast<const char*>(A.in) + off, p, h, A.g.Nh, r);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const uint32_t x = raw_word(r, c);
      const float s = c >= 6 ? al : au;
      acc[c] = {mix_fma<0>(x, s, acc[c].re), mix_fma<1>(x, s, acc[c].im)};
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const char* vb = static_cast<const char*>(A.v[j]) + off + (static_cast<size_t>(p) * 3 * A.g.Nh + h) * 16;
      SpinorRaw<P> v;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const u32x4_t t = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(vb + static_cast<size_t>(k) * A.g.Nh * 16));
        v.b[k] = make_uint4(t.x, t.y, t.z, t.w);
      }
      const float cu = static_cast<float>(A.cv[j]);
      const float cl = ((A.g5v >> j) & 1) ? -cu : cu;
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const uint32_t x = raw_word(v, c);
        const float s = c >= 6 ? cl : cu;
        acc[c] = {mix_fma<0>(x, s, acc[c].re), mix_fma<1>(x, s, acc[c].im)};
      }
    }
  } else {
    Cx<real> s[12];
    SpinorIO<P>::load(static_cast<const char*>(A.in) + off, p, h, A.g.Nh, s);
#pragma unroll
    for (int c = 0; c < 12; ++c) addph<0>(acc[c], s[c], c >= 6 ? al : au);
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      SpinorIO<P>::load_nt(static_cast<const char*>(A.v[j]) + off, p, h, A.g.Nh, s);
      const real cu = static_cast<real>(A.cv[j]);
      const real cl = ((A.g5v >> j) & 1) ? -cu : cu;
#pragma unroll
      for (int c = 0; c < 12; ++c) addph<0>(acc[c], s[c], c >= 6 ? cl : cu);
    }
  }
  SpinorIO<P>::store_nt(static_cast<char*>(A.out) + off, p, h, A.g.Nh, acc);
}

// Site i of logical block lb, for blocks of bs sites: parity p and half
// index h; false past the end.
__device__ inline bool tile_site(const StencilArgs& A, int lb, int bs, int i, int& p, int& h) {
  int hb;
  if (A.npar == 2) {
    p = lb & 1;
    hb = lb >> 1;
  } else {
    p = A.par0;
    hb = lb;
  }
  if (A.tmaj >= 2) {
    // z-slabs of Z = tmaj planes: consecutive blocks cover one slab's
    // (x, y, z) half-slice at t, then the same slab at t + 1, ..., before the
    // next slab, so a site's t-neighbours are read 2 Z Lx Ly / 2 half-sites
    // apart in launch order instead of Lx Ly Lz (a slice of the whole lattice)
    const int Z = A.tmaj, bps = (Z * A.g.sz + bs - 1) / bs;
    const int per_slab = bps * A.g.Lt;
    const int slab = hb / per_slab, r = hb - slab * per_slab;
    const int t = r / bps, j = r - t * bps;
    const int z0 = slab * Z;
    const int len = min(Z, A.g.Lz - z0) * A.g.sz;  // the last slab may be thinner
    const int hl = j * bs + i;
    h = t * A.g.st + z0 * A.g.sz + hl;
    return hl < len;
  }
  if (A.tmaj) {
    const int tile = hb / A.g.Lt, t = hb - tile * A.g.Lt;
    const int hl = tile * bs + i;
    h = t * A.g.st + hl;
    return hl < A.g.st;
  }
  h = hb * bs + i;
  return h < A.g.Nh;
}

// Output site (parity p, half index h) of this thread; false past the end.
__device__ inline bool stencil_site(const StencilArgs& A, int& p, int& h) {
  return tile_site(A, xcd_remap(blockIdx.x, gridDim.x), static_cast<int>(blockDim.x), static_cast<int>(threadIdx.x),
                   p, h);
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
  real bu, bl;
  hop_weights(A, bu, bl);
  hop_dir<P, R, 0, KR, chain_form<P, NV>()>(A, in, p, h, nb, acc, bu, bl);
  hop_dir<P, R, 1, KR, chain_form<P, NV>()>(A, in, p, h, nb, acc, bu, bl);
  hop_dir<P, R, 2, KR, chain_form<P, NV>()>(A, in, p, h, nb, acc, bu, bl);
  hop_dir<P, R, 3, KR, chain_form<P, NV>()>(A, in, p, h, nb, acc, bu, bl);

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
__device__ inline void pipe_consume(const SpinorRaw<P>& sr, const LinkRaw<P, R>& lr, Cx<typename Prec<P>::real>* acc,
                                    typename Prec<P>::real bu, typename Prec<P>::real bl) {
  using real = typename Prec<P>::real;
  constexpr int MU = D / 2;
  constexpr bool CH = P != OVL_F16;  // the pipelined kernels keep the pairwise form for FP16
  Cx<real> hs[2][3], w[2][3], u[3][3];
  link_unpack<P, R>(lr, u);
  opaque_link<P>(u);
  if constexpr (P == OVL_F16) {
    uint32_t sw[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) sw[c] = raw_word(sr, c);
    if constexpr (D % 2 == 0) project_f16<MU, -1>(sw, hs);
    else project_f16<MU, +1>(sw, hs);
  } else {
    Cx<real> s[12];
    spinor_unpack<P>(sr, s);
    if constexpr (D % 2 == 0) project<MU, -1>(s, hs);
    else project<MU, +1>(s, hs);
  }
  if constexpr (D % 2 == 0) {
    colour_mul<false, CH>(u, hs, w);
    accumulate<MU, -1>(acc, w, bu, bl);
  } else {
    colour_mul<true, CH>(u, hs, w);
    accumulate<MU, +1>(acc, w, bu, bl);
  }
}

template <int P, int R, int DEP, int D>
__device__ inline void pipe_run(const StencilArgs& A, const char* in, int p, int h, const int* nb,
                                SpinorRaw<P> (&sr)[DEP], LinkRaw<P, R> (&lr)[DEP],
                                Cx<typename Prec<P>::real>* acc, typename Prec<P>::real bu,
                                typename Prec<P>::real bl) {
  if constexpr (D + DEP - 1 < 8) pipe_issue<P, R, D + DEP - 1>(A, in, p, h, nb, sr[(D + DEP - 1) % DEP], lr[(D + DEP - 1) % DEP]);
  pipe_consume<P, R, D>(sr[D % DEP], lr[D % DEP], acc, bu, bl);
  if constexpr (D + 1 < 8) pipe_run<P, R, DEP, D + 1>(A, in, p, h, nb, sr, lr, acc, bu, bl);
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
  real bu, bl;
  hop_weights(A, bu, bl);
  pipe_run<P, R, DEP, 0>(A, in, p, h, nb, sr, lr, acc, bu, bl);
  epilogue<P, NV>(A, voff, p, h, acc);
}


template <int P, int R, int NV>
void launch_k(const StencilArgs& A0, int nrhs, Shape sh, hipStream_t s) {
  StencilArgs A = A0;
  A.tmaj = sh.tm;
  int hblocks;
  if (sh.tm >= 2) {
    OVL_REQUIRE(sh.tm <= A.g.Lz, OVL_E_ARG, "stencil: slab thicker than the lattice");
    hblocks = ((A.g.Lz + sh.tm - 1) / sh.tm) * A.g.Lt * ((sh.tm * A.g.sz + sh.bs - 1) / sh.bs);
  } else if (sh.tm == 1) {
    hblocks = ((A.g.st + sh.bs - 1) / sh.bs) * A.g.Lt;
  } else {
    hblocks = (A.g.Nh + sh.bs - 1) / sh.bs;
  }
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

}  // namespace
}  // namespace ovl
