// Internal declarations shared by the libovl translation units.
//
// Device-side: complex arithmetic, the 16-byte-block spinor layout for each
// storage precision, the gauge-link layouts (18 or 12 reals), the lattice
// index arithmetic, and the launch helpers.  Host-side: handle structs,
// error reporting and the workspace pool.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <complex>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include <type_traits>

#include "ovl.h"

namespace ovl {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define OVL_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::ovl::Error(OVL_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define OVL_REQUIRE(cond, code, msg)                  \
  do {                                                \
    if (!(cond)) throw ::ovl::Error((code), (msg)); \
  } while (0)

// Runs f() and converts exceptions into ABI status codes.
template <class F>
int guard(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return OVL_E_NOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return OVL_E_ARG;
  }
}

// -------------------------------------------------------------- complex
template <typename T>
struct Cx {
  T re, im;
};

template <typename T>
__host__ __device__ inline Cx<T> cx(T r, T i) {
  return Cx<T>{r, i};
}
template <typename T>
__host__ __device__ inline Cx<T> operator+(Cx<T> a, Cx<T> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename T>
__host__ __device__ inline Cx<T> operator-(Cx<T> a, Cx<T> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename T>
__host__ __device__ inline Cx<T> operator*(Cx<T> a, Cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ inline Cx<T> operator*(T s, Cx<T> a) {
  return {s * a.re, s * a.im};
}
template <typename T>
__host__ __device__ inline Cx<T> conj(Cx<T> a) {
  return {a.re, -a.im};
}
// conj(a) * b
template <typename T>
__host__ __device__ inline Cx<T> cmul_conj(Cx<T> a, Cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i*a and -i*a
template <typename T>
__host__ __device__ inline Cx<T> times_i(Cx<T> a) {
  return {-a.im, a.re};
}
template <typename T>
__host__ __device__ inline Cx<T> times_mi(Cx<T> a) {
  return {a.im, -a.re};
}

// ------------------------------------------------------ storage formats
// A storage format maps 12 complex numbers of compute type `real` to
// 16-byte blocks (spinors) or to K elements of E bytes (links).
struct bf16_t {
  uint16_t bits;
};

__host__ __device__ inline float bf16_to_float(uint16_t b) {
  return __builtin_bit_cast(float, static_cast<uint32_t>(b) << 16);
}
// Round to nearest even; NaN stays a (quiet) NaN.  Written without a branch:
// a data-dependent branch per stored element splits the stencil kernels into
// many basic blocks and the register allocator then keeps every loaded
// neighbour alive across them (256 VGPRs and spills instead of ~80).
__host__ __device__ inline uint16_t float_to_bf16(float f) {
  const uint32_t u = __builtin_bit_cast(uint32_t, f);
  const uint32_t rounded = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  const uint32_t quiet_nan = (u >> 16) | 0x40u;
  return static_cast<uint16_t>(((u & 0x7fffffffu) > 0x7f800000u) ? quiet_nan : rounded);
}

template <int P>
struct Prec;  // P = ovl_prec value

template <>
struct Prec<OVL_F64> {
  using real = double;
  static constexpr int cpb = 1;  // complex per 16-byte block
};
template <>
struct Prec<OVL_F32> {
  using real = float;
  static constexpr int cpb = 2;
};
template <>
struct Prec<OVL_F16> {
  using real = float;
  static constexpr int cpb = 4;
};
template <>
struct Prec<OVL_BF16> {
  using real = float;
  static constexpr int cpb = 4;
};

constexpr int spinor_blocks(int prec) { return prec == OVL_F64 ? 12 : (prec == OVL_F32 ? 6 : 3); }
inline size_t spinor_bytes_per_site(int prec) { return 16u * spinor_blocks(prec); }

// Load/store one 16-byte block as `cpb` complex numbers of compute type.
template <int P>
struct Block;

template <>
struct Block<OVL_F64> {
  __device__ static inline void load(const void* p, Cx<double>* c) {
    double2 v = *reinterpret_cast<const double2*>(p);
    c[0] = {v.x, v.y};
  }
  __device__ static inline void store(void* p, const Cx<double>* c) {
    *reinterpret_cast<double2*>(p) = make_double2(c[0].re, c[0].im);
  }
};
template <>
struct Block<OVL_F32> {
  __device__ static inline void load(const void* p, Cx<float>* c) {
    float4 v = *reinterpret_cast<const float4*>(p);
    c[0] = {v.x, v.y};
    c[1] = {v.z, v.w};
  }
  __device__ static inline void store(void* p, const Cx<float>* c) {
    *reinterpret_cast<float4*>(p) = make_float4(c[0].re, c[0].im, c[1].re, c[1].im);
  }
};
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
template <>
struct Block<OVL_F16> {
  __device__ static inline void load(const void* p, Cx<float>* c) {
    half8_t v = *reinterpret_cast<const half8_t*>(p);
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = {static_cast<float>(v[2 * k]), static_cast<float>(v[2 * k + 1])};
  }
  __device__ static inline void store(void* p, const Cx<float>* c) {
    half8_t v;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[2 * k] = static_cast<_Float16>(c[k].re);
      v[2 * k + 1] = static_cast<_Float16>(c[k].im);
    }
    *reinterpret_cast<half8_t*>(p) = v;
  }
};
template <>
struct Block<OVL_BF16> {
  __device__ static inline void load(const void* p, Cx<float>* c) {
    uint4 v = *reinterpret_cast<const uint4*>(p);
    uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 4; ++k)
      c[k] = {bf16_to_float(static_cast<uint16_t>(w[k] & 0xffffu)),
              bf16_to_float(static_cast<uint16_t>(w[k] >> 16))};
  }
  __device__ static inline void store(void* p, const Cx<float>* c) {
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      w[k] = static_cast<uint32_t>(float_to_bf16(c[k].re)) |
             (static_cast<uint32_t>(float_to_bf16(c[k].im)) << 16);
    *reinterpret_cast<uint4*>(p) = make_uint4(w[0], w[1], w[2], w[3]);
  }
};

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

// One spinor (12 complex) of a field in the [parity][block][Nh] layout.
// `base` points at the start of the vector, `h` is the half-lattice index,
// `p` the parity.
template <int P>
struct SpinorIO {
  using real = typename Prec<P>::real;
  static constexpr int cpb = Prec<P>::cpb;
  static constexpr int nb = 12 / cpb;
  __device__ static inline void load(const void* base, int p, int h, int Nh, Cx<real>* s) {
    const char* b = static_cast<const char*>(base) + (static_cast<size_t>(p) * nb * Nh + h) * 16;
#pragma unroll
    for (int j = 0; j < nb; ++j) Block<P>::load(b + static_cast<size_t>(j) * Nh * 16, s + j * cpb);
  }
  __device__ static inline void store(void* base, int p, int h, int Nh, const Cx<real>* s) {
    char* b = static_cast<char*>(base) + (static_cast<size_t>(p) * nb * Nh + h) * 16;
#pragma unroll
    for (int j = 0; j < nb; ++j) Block<P>::store(b + static_cast<size_t>(j) * Nh * 16, s + j * cpb);
  }
  // Streaming variants for data touched once per launch (epilogue vectors,
  // the output): non-temporal, so they do not displace the neighbour and
  // link lines the stencil reuses from L2.
  __device__ static inline void load_nt(const void* base, int p, int h, int Nh, Cx<real>* s) {
    const char* b = static_cast<const char*>(base) + (static_cast<size_t>(p) * nb * Nh + h) * 16;
#pragma unroll
    for (int j = 0; j < nb; ++j) {
      const u32x4_t v = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(b + static_cast<size_t>(j) * Nh * 16));
      Block<P>::load(&v, s + j * cpb);
    }
  }
  __device__ static inline void store_nt(void* base, int p, int h, int Nh, const Cx<real>* s) {
    char* b = static_cast<char*>(base) + (static_cast<size_t>(p) * nb * Nh + h) * 16;
#pragma unroll
    for (int j = 0; j < nb; ++j) {
      u32x4_t v;
      Block<P>::store(&v, s + j * cpb);
      __builtin_nontemporal_store(v, reinterpret_cast<u32x4_t*>(b + static_cast<size_t>(j) * Nh * 16));
    }
  }
};

// Raw (still encoded) spinor: its 16-byte blocks, for loads issued ahead of
// the arithmetic that consumes them.
template <int P>
struct SpinorRaw {
  uint4 b[12 / Prec<P>::cpb];
};

template <int P>
__device__ inline void spinor_load_raw(const void* base, int p, int h, int Nh, SpinorRaw<P>& r) {
  constexpr int nb = 12 / Prec<P>::cpb;
  const char* b = static_cast<const char*>(base) + (static_cast<size_t>(p) * nb * Nh + h) * 16;
#pragma unroll
  for (int j = 0; j < nb; ++j) r.b[j] = *reinterpret_cast<const uint4*>(b + static_cast<size_t>(j) * Nh * 16);
}

template <int P>
__device__ inline void spinor_unpack(const SpinorRaw<P>& r, Cx<typename Prec<P>::real>* s) {
  constexpr int cpb = Prec<P>::cpb;
#pragma unroll
  for (int j = 0; j < 12 / cpb; ++j) Block<P>::load(&r.b[j], s + j * cpb);
}

// ------------------------------------------------------------ link formats
// Layout [mu][parity][K][Nh] of E-byte elements.  R = 18 or 12 reals.
//   F64: E = 16 (one complex);            K = 9 or 6
//   F32: R=18 -> E = 8 (one complex),     K = 9;  R=12 -> E = 16 (two), K = 3
//   F16/BF16: R=18 -> E = 4 (one complex), K = 9; R=12 -> E = 8 (two), K = 3
template <int P, int R>
struct LinkFmt {
  static constexpr int ncx = R / 2;  // stored complex numbers
  static constexpr int cpe = (P == OVL_F64 || R == 18) ? 1 : 2;  // complex per element
  static constexpr int K = ncx / cpe;
  static constexpr int E = (P == OVL_F64 ? 16 : (P == OVL_F32 ? 8 : 4)) * cpe;
};

template <int P>
struct ScalarIO;
template <>
struct ScalarIO<OVL_F64> {
  __device__ static inline Cx<double> load1(const char* p) {
    double2 v = *reinterpret_cast<const double2*>(p);
    return {v.x, v.y};
  }
  __device__ static inline void load2(const char* p, Cx<double>* c) {
    c[0] = load1(p);
    c[1] = load1(p + 16);
  }
  __device__ static inline void store1(char* p, Cx<double> c) {
    *reinterpret_cast<double2*>(p) = make_double2(c.re, c.im);
  }
};
template <>
struct ScalarIO<OVL_F32> {
  __device__ static inline Cx<float> load1(const char* p) {
    float2 v = *reinterpret_cast<const float2*>(p);
    return {v.x, v.y};
  }
  __device__ static inline void load2(const char* p, Cx<float>* c) {
    float4 v = *reinterpret_cast<const float4*>(p);
    c[0] = {v.x, v.y};
    c[1] = {v.z, v.w};
  }
  __device__ static inline void store1(char* p, Cx<float> c) {
    *reinterpret_cast<float2*>(p) = make_float2(c.re, c.im);
  }
  __device__ static inline void store2(char* p, const Cx<float>* c) {
    *reinterpret_cast<float4*>(p) = make_float4(c[0].re, c[0].im, c[1].re, c[1].im);
  }
};
typedef _Float16 half2v_t __attribute__((ext_vector_type(2)));
typedef _Float16 half4v_t __attribute__((ext_vector_type(4)));
template <>
struct ScalarIO<OVL_F16> {
  __device__ static inline Cx<float> load1(const char* p) {
    half2v_t v = *reinterpret_cast<const half2v_t*>(p);
    return {static_cast<float>(v[0]), static_cast<float>(v[1])};
  }
  __device__ static inline void load2(const char* p, Cx<float>* c) {
    half4v_t v = *reinterpret_cast<const half4v_t*>(p);
    c[0] = {static_cast<float>(v[0]), static_cast<float>(v[1])};
    c[1] = {static_cast<float>(v[2]), static_cast<float>(v[3])};
  }
  __device__ static inline void store1(char* p, Cx<float> c) {
    half2v_t v;
    v[0] = static_cast<_Float16>(c.re);
    v[1] = static_cast<_Float16>(c.im);
    *reinterpret_cast<half2v_t*>(p) = v;
  }
  __device__ static inline void store2(char* p, const Cx<float>* c) {
    half4v_t v;
    v[0] = static_cast<_Float16>(c[0].re);
    v[1] = static_cast<_Float16>(c[0].im);
    v[2] = static_cast<_Float16>(c[1].re);
    v[3] = static_cast<_Float16>(c[1].im);
    *reinterpret_cast<half4v_t*>(p) = v;
  }
};
template <>
struct ScalarIO<OVL_BF16> {
  __device__ static inline Cx<float> load1(const char* p) {
    uint32_t w = *reinterpret_cast<const uint32_t*>(p);
    return {bf16_to_float(static_cast<uint16_t>(w & 0xffffu)), bf16_to_float(static_cast<uint16_t>(w >> 16))};
  }
  __device__ static inline void load2(const char* p, Cx<float>* c) {
    uint2 w = *reinterpret_cast<const uint2*>(p);
    c[0] = {bf16_to_float(static_cast<uint16_t>(w.x & 0xffffu)), bf16_to_float(static_cast<uint16_t>(w.x >> 16))};
    c[1] = {bf16_to_float(static_cast<uint16_t>(w.y & 0xffffu)), bf16_to_float(static_cast<uint16_t>(w.y >> 16))};
  }
  __device__ static inline void store1(char* p, Cx<float> c) {
    *reinterpret_cast<uint32_t*>(p) =
        static_cast<uint32_t>(float_to_bf16(c.re)) | (static_cast<uint32_t>(float_to_bf16(c.im)) << 16);
  }
  __device__ static inline void store2(char* p, const Cx<float>* c) {
    uint2 w;
    w.x = static_cast<uint32_t>(float_to_bf16(c[0].re)) | (static_cast<uint32_t>(float_to_bf16(c[0].im)) << 16);
    w.y = static_cast<uint32_t>(float_to_bf16(c[1].re)) | (static_cast<uint32_t>(float_to_bf16(c[1].im)) << 16);
    *reinterpret_cast<uint2*>(p) = w;
  }
};

template <typename T>
__host__ __device__ inline T ffma(T a, T b, T c) {
  if constexpr (std::is_same_v<T, double>)
    return __builtin_fma(a, b, c);
  else
    return __builtin_fmaf(a, b, c);
}

// Third row of an SU(3) matrix from the first two: row2 = conj(row0 x row1).
// Element c is conj(x y - z w) with x = r0[a], y = r1[b], z = r0[b],
// w = r1[a] and (a, b) the two columns after c (cyclically), four FMAs for
// each real part.
template <typename T>
__device__ inline void reconstruct_row2(Cx<T> (*u)[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    const Cx<T> x = u[0][a], y = u[1][b], z = u[0][b], w = u[1][a];
    T re = x.re * y.re;
    re = ffma(-x.im, y.im, re);
    re = ffma(-z.re, w.re, re);
    re = ffma(z.im, w.im, re);
    T im = z.re * w.im;  // imaginary part of the conjugate
    im = ffma(z.im, w.re, im);
    im = ffma(-x.re, y.im, im);
    im = ffma(-x.im, y.re, im);
    u[2][c] = {re, im};
  }
}

// Loads the 3x3 link matrix u[row][col] of direction mu at (p, h).
template <int P, int R>
struct LinkIO {
  using F = LinkFmt<P, R>;
  using real = typename Prec<P>::real;
  __device__ static inline void load(const void* links, int mu, int p, int h, int Nh, Cx<real> (*u)[3]) {
    const char* b = static_cast<const char*>(links) +
                    ((static_cast<size_t>(mu) * 2 + p) * F::K * Nh + h) * F::E;
    Cx<real> c[9];
    if constexpr (F::cpe == 1) {
#pragma unroll
      for (int k = 0; k < F::ncx; ++k) c[k] = ScalarIO<P>::load1(b + static_cast<size_t>(k) * Nh * F::E);
    } else {
#pragma unroll
      for (int k = 0; k < F::K; ++k) ScalarIO<P>::load2(b + static_cast<size_t>(k) * Nh * F::E, c + 2 * k);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) u[k / 3][k % 3] = c[k];
    if constexpr (R == 18) {
#pragma unroll
      for (int k = 6; k < 9; ++k) u[2][k - 6] = c[k];
    } else {
      reconstruct_row2(u);
    }
  }
};

// Raw (still encoded) link: K elements of E bytes as 32-bit words.
template <int P, int R>
struct LinkRaw {
  using F = LinkFmt<P, R>;
  uint32_t w[F::K * F::E / 4];
};

template <int P, int R>
__device__ inline void link_load_raw(const void* links, int mu, int p, int h, int Nh, LinkRaw<P, R>& r) {
  using F = LinkFmt<P, R>;
  const char* b = static_cast<const char*>(links) + ((static_cast<size_t>(mu) * 2 + p) * F::K * Nh + h) * F::E;
#pragma unroll
  for (int k = 0; k < F::K; ++k) {
    const char* a = b + static_cast<size_t>(k) * Nh * F::E;
    if constexpr (F::E == 16) {
      const uint4 v = *reinterpret_cast<const uint4*>(a);
      r.w[4 * k] = v.x;
      r.w[4 * k + 1] = v.y;
      r.w[4 * k + 2] = v.z;
      r.w[4 * k + 3] = v.w;
    } else if constexpr (F::E == 8) {
      const uint2 v = *reinterpret_cast<const uint2*>(a);
      r.w[2 * k] = v.x;
      r.w[2 * k + 1] = v.y;
    } else {
      r.w[k] = *reinterpret_cast<const uint32_t*>(a);
    }
  }
}

template <int P, int R>
__device__ inline void link_unpack(const LinkRaw<P, R>& r, Cx<typename Prec<P>::real> (*u)[3]) {
  using F = LinkFmt<P, R>;
  using real = typename Prec<P>::real;
  const char* b = reinterpret_cast<const char*>(r.w);
  Cx<real> c[9];
  if constexpr (F::cpe == 1) {
#pragma unroll
    for (int k = 0; k < F::ncx; ++k) c[k] = ScalarIO<P>::load1(b + k * F::E);
  } else {
#pragma unroll
    for (int k = 0; k < F::K; ++k) ScalarIO<P>::load2(b + k * F::E, c + 2 * k);
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) u[k / 3][k % 3] = c[k];
  if constexpr (R == 18) {
#pragma unroll
    for (int k = 6; k < 9; ++k) u[2][k - 6] = c[k];
  } else {
    reconstruct_row2(u);
  }
}

// ------------------------------------------------------------ geometry
struct Geo {
  int Lx, Ly, Lz, Lt;
  int lxh;       // Lx / 2
  int Nh;        // N / 2
  int sy, sz, st;  // half-index strides of y, z, t
};

// Coordinates of half-index h at parity p.
__host__ __device__ inline void site_coords(const Geo& g, int p, int h, int& x, int& y, int& z, int& t) {
  int xh = h % g.lxh;
  int r = h / g.lxh;
  y = r % g.Ly;
  r /= g.Ly;
  z = r % g.Lz;
  t = r / g.Lz;
  x = 2 * xh + ((p + y + z + t) & 1);
}

// Half-index of the 8 neighbours (all of parity 1-p), order +x,+y,+z,+t,-x,-y,-z,-t.
__host__ __device__ inline void site_neighbors(const Geo& g, int h, int x, int y, int z, int t, int* nb) {
  const int base = h - (x >> 1);  // h with the x part removed
  int xp = (x + 1 == g.Lx) ? 0 : x + 1;
  int xm = (x == 0) ? g.Lx - 1 : x - 1;
  nb[0] = base + (xp >> 1);
  nb[4] = base + (xm >> 1);
  nb[1] = h + ((y + 1 == g.Ly) ? -(g.Ly - 1) * g.sy : g.sy);
  nb[5] = h + ((y == 0) ? (g.Ly - 1) * g.sy : -g.sy);
  nb[2] = h + ((z + 1 == g.Lz) ? -(g.Lz - 1) * g.sz : g.sz);
  nb[6] = h + ((z == 0) ? (g.Lz - 1) * g.sz : -g.sz);
  nb[3] = h + ((t + 1 == g.Lt) ? -(g.Lt - 1) * g.st : g.st);
  nb[7] = h + ((t == 0) ? (g.Lt - 1) * g.st : -g.st);
}

// XCD-aware block remap: hardware hands workgroups to the 8 XCDs round
// robin; this makes each XCD take one contiguous range of logical blocks so
// that neighbouring sites share an L2.
__device__ inline int xcd_remap(int b, int nblocks) {
  constexpr int NX = 8;
  int q = nblocks / NX, r = nblocks % NX;
  int x = b % NX, j = b / NX;
  return x * q + (x < r ? x : r) + j;
}

// ------------------------------------------------------------- handles
}  // namespace ovl

struct ovl_geom {
  int dims[4];
  int64_t N;
  ovl::Geo geo;
};

struct ovl_gauge {
  ovl_geom geom;             // the handle keeps its own copy of the geometry
  void* master = nullptr;    // FP64, 18 reals: source of every representation
  void* links[4] = {nullptr, nullptr, nullptr, nullptr};  // used per spinor precision
  int recon[4] = {0, 0, 0, 0};                             // 18 or 12 (0 = absent)
};

struct ovl_sign {
  double lam_max;
  double eps;
  double delta;           // measured max |1 - sqrt(x) P(x)| on [eps, 1]
  std::vector<double> c;  // c_0..c_n, c_0 already halved
};

struct ovl_lowmodes {
  ovl_geom geom;
  int ell;
  const void* V;  // borrowed: ell FP64 spinors
  std::vector<double> lambda;
  double* dev_sign = nullptr;  // sign(lambda_i) on the device
};

// Eigenpairs of the massless overlap operator used to deflate D(m) (eq. 9).
struct ovl_deflation {
  ovl_geom geom;
  int n;
  const void* Xi;                       // borrowed: n FP64 spinors
  std::vector<std::complex<double>> d;  // eigenvalues of D
  // minimal-residual form (after ovl_deflation_prepare): Z = D(0) Xi
  // (borrowed, n FP64 spinors) for the rho it was made with, and the Gram
  // matrices ZZ = Z^dag Z, ZX = Z^dag Xi, XX = Xi^dag Xi (column-major n x n)
  const void* Z = nullptr;
  double rho = 0.0;
  std::vector<std::complex<double>> ZZ, ZX, XX;
};

struct ovl_net {
  ovl_geom geom;
  int hidden;
  // host FP64 weights, layout [k][a][b][s][t] complex
  std::vector<std::complex<double>> w1, w2;  // 9 x hidden x 1 x 16, 9 x 1 x hidden x 16
};

namespace ovl {

// Device workspace pool.  A buffer released on stream s is only handed out
// again for work on the same stream, so stream order makes reuse safe even
// while earlier kernels that used it are still running.
void* ws_get(size_t bytes, hipStream_t s);
void ws_put(void* p, hipStream_t s);
// Hands every free buffer keyed by stream `from` over to stream `to`.  Safe
// when `to` is ordered after all work queued on `from` so far (an event
// wait, or a synchronize of `from`).  The solvers run on private streams:
// they adopt the caller's free buffers at the start and hand theirs back
// at the end, so repeated solves reuse one set of buffers and none is left
// under a dead stream handle.
void ws_retire_stream(hipStream_t from, hipStream_t to);
// Accounting of the device memory the library holds (workspace pool,
// eigensolver buffers, packed links): +bytes on allocation, -bytes on free.
void mem_track(int64_t delta);
// OVL_LOG=1 in the environment: the solvers print one line per outer cycle
// (and the CG every 100 inner iterations) on stderr.
bool log_on();

struct WsBuf {
  void* p = nullptr;
  hipStream_t s;
  WsBuf(size_t bytes, hipStream_t st) : p(ws_get(bytes, st)), s(st) {}
  ~WsBuf() { ws_put(p, s); }
  WsBuf(const WsBuf&) = delete;
  WsBuf& operator=(const WsBuf&) = delete;
};

inline size_t spinor_vec_bytes(const ovl_geom* g, int prec) {
  return static_cast<size_t>(g->N) * spinor_bytes_per_site(prec);
}

void check_prec(int prec);
void check_nrhs(int nrhs);

}  // namespace ovl
