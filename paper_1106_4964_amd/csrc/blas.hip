// Vector operations and reductions (arXiv:1106.4964 Sec. III: the local
// vector operations and the scalar product / norm that the solvers use).
//
// Every kernel walks a vector as 16-byte blocks, so one thread moves one
// fully coalesced 16-byte load per operand whatever the storage precision.
// Reductions accumulate in FP64: each block of a fixed-size grid reduces its
// grid-stride share with wave64 shuffles and LDS, and a second one-block
// kernel adds the per-block partials in a fixed order, so a given input
// always gives the same bits.
#include <type_traits>

#include "ops.h"

namespace ovl {
namespace {

constexpr int RED_BLOCKS = 1024;
constexpr int RED_THREADS = 256;

template <int P>
__global__ void axpy_kernel(size_t n16, const double* a, const char* x, char* y, size_t vstride) {
  using real = typename Prec<P>::real;
  constexpr int cpb = Prec<P>::cpb;
  const size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (i >= n16) return;
  const size_t off = blockIdx.y * vstride + i * 16;
  const Cx<real> ar = {static_cast<real>(a[2 * blockIdx.y]), static_cast<real>(a[2 * blockIdx.y + 1])};
  Cx<real> xv[cpb], yv[cpb];
  Block<P>::load(x + off, xv);
  Block<P>::load(y + off, yv);
#pragma unroll
  for (int k = 0; k < cpb; ++k) yv[k] = yv[k] + ar * xv[k];
  Block<P>::store(y + off, yv);
}

template <int P>
__global__ void xpay_kernel(size_t n16, const char* x, const double* a, char* y, size_t vstride) {
  using real = typename Prec<P>::real;
  constexpr int cpb = Prec<P>::cpb;
  const size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (i >= n16) return;
  const size_t off = blockIdx.y * vstride + i * 16;
  const Cx<real> ar = {static_cast<real>(a[2 * blockIdx.y]), static_cast<real>(a[2 * blockIdx.y + 1])};
  Cx<real> xv[cpb], yv[cpb];
  Block<P>::load(x + off, xv);
  Block<P>::load(y + off, yv);
#pragma unroll
  for (int k = 0; k < cpb; ++k) yv[k] = xv[k] + ar * yv[k];
  Block<P>::store(y + off, yv);
}

// Precision conversion, one thread per site (the block layouts differ
// between precisions, so whole spinors are moved).
template <int PS, int PD>
__global__ void convert_kernel(int Nh, const char* src, char* dst, size_t sstride, size_t dstride) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * Nh) return;
  const int p = e >= Nh, h = e - p * Nh;
  using rs = typename Prec<PS>::real;
  using rd = typename Prec<PD>::real;
  Cx<rs> a[12];
  SpinorIO<PS>::load(src + blockIdx.y * sstride, p, h, Nh, a);
  Cx<rd> b[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) b[k] = {static_cast<rd>(a[k].re), static_cast<rd>(a[k].im)};
  SpinorIO<PD>::store(dst + blockIdx.y * dstride, p, h, Nh, b);
}

// out = gamma5 in: complex index c = 3*spin + colour, spins 2 and 3 negated.
// In place: keep the chirality sector[r] (+1: spins 0, 1; -1: spins 2, 3)
// of vector r, zero the other; sector 0 leaves the vector unchanged.
template <int P>
__global__ void chiral_kernel(size_t n16, int Nh, char* x, size_t vstride, const int* sector) {
  using real = typename Prec<P>::real;
  constexpr int cpb = Prec<P>::cpb;
  const size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  const int sc = sector[blockIdx.y];
  if (i >= n16 || sc == 0) return;
  const size_t off = blockIdx.y * vstride + i * 16;
  const int j = static_cast<int>((i / Nh) % (12 / cpb));
  Cx<real> v[cpb];
  Block<P>::load(x + off, v);
#pragma unroll
  for (int k = 0; k < cpb; ++k) {
    const bool upper = j * cpb + k < 6;
    if (upper != (sc > 0)) v[k] = {real(0), real(0)};
  }
  Block<P>::store(x + off, v);
}

template <int P>
__global__ void gamma5_kernel(size_t n16, int Nh, const char* x, char* y, size_t vstride) {
  using real = typename Prec<P>::real;
  constexpr int cpb = Prec<P>::cpb;
  const size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (i >= n16) return;
  const size_t off = blockIdx.y * vstride + i * 16;
  const int j = static_cast<int>((i / Nh) % (12 / cpb));  // block index within the site
  Cx<real> v[cpb];
  Block<P>::load(x + off, v);
#pragma unroll
  for (int k = 0; k < cpb; ++k)
    if (j * cpb + k >= 6) v[k] = real(-1) * v[k];
  Block<P>::store(y + off, v);
}

// y(PY) = a x(PX) + b y(PY), per site, with complex a, b per rhs read from
// device memory (a[2r], a[2r+1]); y is not read when READY is false.
template <int PX, int PY, bool READY>
__global__ void axpby_kernel(int Nh, const double* a, const char* x, const double* b, char* y, size_t sx,
                             size_t sy) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * Nh) return;
  const int p = e >= Nh, h = e - p * Nh, r = blockIdx.y;
  using rx = typename Prec<PX>::real;
  using ry = typename Prec<PY>::real;
  using rc = typename std::conditional<(sizeof(rx) > sizeof(ry)), rx, ry>::type;
  Cx<rx> xv[12];
  SpinorIO<PX>::load(x + r * sx, p, h, Nh, xv);
  const Cx<rc> ar = {static_cast<rc>(a[2 * r]), static_cast<rc>(a[2 * r + 1])};
  Cx<ry> out[12];
  if constexpr (READY) {
    Cx<ry> yv[12];
    SpinorIO<PY>::load(y + r * sy, p, h, Nh, yv);
    const Cx<rc> br = {static_cast<rc>(b[2 * r]), static_cast<rc>(b[2 * r + 1])};
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const Cx<rc> xx = {static_cast<rc>(xv[k].re), static_cast<rc>(xv[k].im)};
      const Cx<rc> yy = {static_cast<rc>(yv[k].re), static_cast<rc>(yv[k].im)};
      const Cx<rc> z = ar * xx + br * yy;
      out[k] = {static_cast<ry>(z.re), static_cast<ry>(z.im)};
    }
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const Cx<rc> xx = {static_cast<rc>(xv[k].re), static_cast<rc>(xv[k].im)};
      const Cx<rc> z = ar * xx;
      out[k] = {static_cast<ry>(z.re), static_cast<ry>(z.im)};
    }
  }
  SpinorIO<PY>::store(y + r * sy, p, h, Nh, out);
}

// y = 0 (a fill kernel, so that it can live inside a captured graph)
__global__ void zero_kernel(size_t n16, uint4* y) {
  const size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (i < n16) y[i] = make_uint4(0u, 0u, 0u, 0u);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block sum of (re, im) pairs; result valid in thread 0.
__device__ inline void block_sum2(double& re, double& im) {
  __shared__ double sre[RED_THREADS / 64], sim[RED_THREADS / 64];
  re = wave_sum(re);
  im = wave_sum(im);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sre[w] = re;
    sim[w] = im;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    re = 0.0;
    im = 0.0;
    for (int k = 0; k < RED_THREADS / 64; ++k) {
      re += sre[k];
      im += sim[k];
    }
  }
}

template <int P, bool NORM>
__global__ __launch_bounds__(RED_THREADS) void dot_partial_kernel(size_t n16, const char* x, const char* y,
                                                                  size_t vstride, double* partial) {
  using real = typename Prec<P>::real;
  constexpr int cpb = Prec<P>::cpb;
  double re = 0.0, im = 0.0;
  const char* xb = x + blockIdx.y * vstride;
  const char* yb = NORM ? xb : y + blockIdx.y * vstride;
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n16;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    Cx<real> xv[cpb];
    Block<P>::load(xb + i * 16, xv);
    if constexpr (NORM) {
#pragma unroll
      for (int k = 0; k < cpb; ++k) {
        re += static_cast<double>(xv[k].re) * xv[k].re;
        re += static_cast<double>(xv[k].im) * xv[k].im;
      }
    } else {
      Cx<real> yv[cpb];
      Block<P>::load(yb + i * 16, yv);
#pragma unroll
      for (int k = 0; k < cpb; ++k) {
        const double xr = xv[k].re, xi = xv[k].im, yr = yv[k].re, yi = yv[k].im;
        re += xr * yr + xi * yi;
        im += xr * yi - xi * yr;
      }
    }
  }
  block_sum2(re, im);
  if (threadIdx.x == 0) {
    double* o = partial + (static_cast<size_t>(blockIdx.y) * gridDim.x + blockIdx.x) * 2;
    o[0] = re;
    o[1] = im;
  }
}

// One block per rhs: fixed-order sum of the RED_BLOCKS partials.
__global__ __launch_bounds__(RED_THREADS) void dot_final_kernel(const double* partial, int nparts, double* out) {
  double re = 0.0, im = 0.0;
  const double* p = partial + static_cast<size_t>(blockIdx.x) * nparts * 2;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    re += p[2 * i];
    im += p[2 * i + 1];
  }
  block_sum2(re, im);
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = re;
    out[2 * blockIdx.x + 1] = im;
  }
}

template <template <int> class K, typename... Args>
void dispatch_prec(int prec, Args&&... args) {
  switch (prec) {
    case OVL_F64: K<OVL_F64>::run(args...); break;
    case OVL_F32: K<OVL_F32>::run(args...); break;
    case OVL_F16: K<OVL_F16>::run(args...); break;
    case OVL_BF16: K<OVL_BF16>::run(args...); break;
    default: throw Error(OVL_E_PRECISION, "unknown precision");
  }
}

template <int P>
struct AxpyL {
  static void run(size_t n16, const double* a, const void* x, void* y, int nrhs, size_t vs, hipStream_t s) {
    dim3 grid((n16 + 255) / 256, nrhs);
    hipLaunchKernelGGL(axpy_kernel<P>, grid, dim3(256), 0, s, n16, a, static_cast<const char*>(x),
                       static_cast<char*>(y), vs);
  }
};
template <int P>
struct XpayL {
  static void run(size_t n16, const void* x, const double* a, void* y, int nrhs, size_t vs, hipStream_t s) {
    dim3 grid((n16 + 255) / 256, nrhs);
    hipLaunchKernelGGL(xpay_kernel<P>, grid, dim3(256), 0, s, n16, static_cast<const char*>(x), a,
                       static_cast<char*>(y), vs);
  }
};
template <int P>
struct G5L {
  static void run(size_t n16, int Nh, const void* x, void* y, int nrhs, size_t vs, hipStream_t s) {
    dim3 grid((n16 + 255) / 256, nrhs);
    hipLaunchKernelGGL(gamma5_kernel<P>, grid, dim3(256), 0, s, n16, Nh, static_cast<const char*>(x),
                       static_cast<char*>(y), vs);
  }
};
template <int P>
struct ChiralL {
  static void run(size_t n16, int Nh, void* x, int nrhs, size_t vs, const int* sector, hipStream_t s) {
    dim3 grid((n16 + 255) / 256, nrhs);
    hipLaunchKernelGGL(chiral_kernel<P>, grid, dim3(256), 0, s, n16, Nh, static_cast<char*>(x), vs, sector);
  }
};
template <int P>
struct DotL {
  static void run(size_t n16, const void* x, const void* y, int nrhs, size_t vs, double* out, hipStream_t s) {
    WsBuf part(static_cast<size_t>(nrhs) * RED_BLOCKS * 2 * sizeof(double), s);
    double* pp = static_cast<double*>(part.p);
    if (y)
      hipLaunchKernelGGL((dot_partial_kernel<P, false>), dim3(RED_BLOCKS, nrhs), dim3(RED_THREADS), 0, s, n16,
                         static_cast<const char*>(x), static_cast<const char*>(y), vs, pp);
    else
      hipLaunchKernelGGL((dot_partial_kernel<P, true>), dim3(RED_BLOCKS, nrhs), dim3(RED_THREADS), 0, s, n16,
                         static_cast<const char*>(x), nullptr, vs, pp);
    hipLaunchKernelGGL(dot_final_kernel, dim3(nrhs), dim3(RED_THREADS), 0, s, pp, RED_BLOCKS, out);
  }
};

template <int PS>
struct ConvL {
  template <int PD>
  static void go(int Nh, const void* src, void* dst, int nrhs, hipStream_t s) {
    const size_t ss = static_cast<size_t>(2) * Nh * spinor_bytes_per_site(PS);
    const size_t ds = static_cast<size_t>(2) * Nh * spinor_bytes_per_site(PD);
    dim3 grid((2 * Nh + 255) / 256, nrhs);
    hipLaunchKernelGGL((convert_kernel<PS, PD>), grid, dim3(256), 0, s, Nh, static_cast<const char*>(src),
                       static_cast<char*>(dst), ss, ds);
  }
  static void run(int dprec, int Nh, const void* src, void* dst, int nrhs, hipStream_t s) {
    switch (dprec) {
      case OVL_F64: go<OVL_F64>(Nh, src, dst, nrhs, s); break;
      case OVL_F32: go<OVL_F32>(Nh, src, dst, nrhs, s); break;
      case OVL_F16: go<OVL_F16>(Nh, src, dst, nrhs, s); break;
      case OVL_BF16: go<OVL_BF16>(Nh, src, dst, nrhs, s); break;
      default: throw Error(OVL_E_PRECISION, "unknown precision");
    }
  }
};

}  // namespace

void blas_axpy(int prec, size_t n16, const double* a, const void* x, void* y, int nrhs, size_t vstride,
               hipStream_t s) {
  dispatch_prec<AxpyL>(prec, n16, a, x, y, nrhs, vstride, s);
  OVL_HIP(hipGetLastError());
}

void blas_xpay(int prec, size_t n16, const void* x, const double* a, void* y, int nrhs, size_t vstride,
               hipStream_t s) {
  dispatch_prec<XpayL>(prec, n16, x, a, y, nrhs, vstride, s);
  OVL_HIP(hipGetLastError());
}

template <int PX, int PY>
void axpby_go(int Nh, const double* a, const void* x, const double* b, void* y, int nrhs, hipStream_t s) {
  const size_t sx = static_cast<size_t>(2) * Nh * spinor_bytes_per_site(PX);
  const size_t sy = static_cast<size_t>(2) * Nh * spinor_bytes_per_site(PY);
  dim3 grid((2 * Nh + 255) / 256, nrhs);
  if (b)
    hipLaunchKernelGGL((axpby_kernel<PX, PY, true>), grid, dim3(256), 0, s, Nh, a, static_cast<const char*>(x), b,
                       static_cast<char*>(y), sx, sy);
  else
    hipLaunchKernelGGL((axpby_kernel<PX, PY, false>), grid, dim3(256), 0, s, Nh, a, static_cast<const char*>(x),
                       b, static_cast<char*>(y), sx, sy);
}

template <int PX>
void axpby_py(int py, int Nh, const double* a, const void* x, const double* b, void* y, int nrhs, hipStream_t s) {
  switch (py) {
    case OVL_F64: axpby_go<PX, OVL_F64>(Nh, a, x, b, y, nrhs, s); break;
    case OVL_F32: axpby_go<PX, OVL_F32>(Nh, a, x, b, y, nrhs, s); break;
    case OVL_F16: axpby_go<PX, OVL_F16>(Nh, a, x, b, y, nrhs, s); break;
    case OVL_BF16: axpby_go<PX, OVL_BF16>(Nh, a, x, b, y, nrhs, s); break;
    default: throw Error(OVL_E_PRECISION, "unknown precision");
  }
}

void blas_axpby(int px, const void* x, const double* a, int py, void* y, const double* b, size_t nsites, int nrhs,
                hipStream_t s) {
  const int Nh = static_cast<int>(nsites / 2);
  switch (px) {
    case OVL_F64: axpby_py<OVL_F64>(py, Nh, a, x, b, y, nrhs, s); break;
    case OVL_F32: axpby_py<OVL_F32>(py, Nh, a, x, b, y, nrhs, s); break;
    case OVL_F16: axpby_py<OVL_F16>(py, Nh, a, x, b, y, nrhs, s); break;
    case OVL_BF16: axpby_py<OVL_BF16>(py, Nh, a, x, b, y, nrhs, s); break;
    default: throw Error(OVL_E_PRECISION, "unknown precision");
  }
  OVL_HIP(hipGetLastError());
}

void blas_zero(void* y, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  hipLaunchKernelGGL(zero_kernel, dim3((n16 + 255) / 256), dim3(256), 0, s, n16, static_cast<uint4*>(y));
  OVL_HIP(hipGetLastError());
}

void blas_chiral(int prec, size_t vstride, void* x, int nrhs, const int* dev_sector, hipStream_t s) {
  const size_t n16 = vstride / 16;
  const int Nh = static_cast<int>(n16 / (2 * spinor_blocks(prec)));
  dispatch_prec<ChiralL>(prec, n16, Nh, x, nrhs, vstride, dev_sector, s);
  OVL_HIP(hipGetLastError());
}

void blas_gamma5(int prec, size_t vstride, const void* x, void* y, int nrhs, hipStream_t s) {
  const size_t n16 = vstride / 16;
  const int Nh = static_cast<int>(n16 / (2 * spinor_blocks(prec)));
  dispatch_prec<G5L>(prec, n16, Nh, x, y, nrhs, vstride, s);
  OVL_HIP(hipGetLastError());
}

void blas_dot(int prec, size_t n16, const void* x, const void* y, int nrhs, size_t vstride, double* dev_out,
              hipStream_t s) {
  dispatch_prec<DotL>(prec, n16, x, y, nrhs, vstride, dev_out, s);
  OVL_HIP(hipGetLastError());
}

void blas_norm2(int prec, size_t n16, const void* x, int nrhs, size_t vstride, double* dev_out, hipStream_t s) {
  dispatch_prec<DotL>(prec, n16, x, static_cast<const void*>(nullptr), nrhs, vstride, dev_out, s);
  OVL_HIP(hipGetLastError());
}

void blas_convert(int sprec, const void* src, int dprec, void* dst, size_t nsites, int nrhs, hipStream_t s) {
  dispatch_prec<ConvL>(sprec, dprec, static_cast<int>(nsites / 2), src, dst, nrhs, s);
  OVL_HIP(hipGetLastError());
}

}  // namespace ovl
