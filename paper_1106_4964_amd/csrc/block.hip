// Tall-skinny block operations between a set of FP64 basis vectors V
// (eigenvectors, Krylov or subspace bases) and a batch of R <= 12 spinors:
//
//   block_dot   : C[i][r] = V_i^dag psi_r             (FP64 accumulation)
//   block_axpy  : Y_r     = [Y_r] + sum_i V_i K[i][r]
//   lowmode_project (eq. 6-7 of arXiv:1106.4964):
//       psi_h = psi - sum_i (V_i^dag psi) V_i,
//       w     = [gamma5] sum_i sign(lambda_i) (V_i^dag psi) V_i
//
// Both sweeps read V exactly once.  Elements are walked in "rows"
// (parity p, complex index c) of N/2 sites, so a complex number is addressed
// the same way whatever the storage precision of the batch.
//
// block_dot is a split-K product: each block of a 512-block grid takes a
// contiguous range of 64-element tiles, stages the batch tile in LDS, and
// every wave accumulates IW basis vectors against it in registers; a second
// kernel adds the per-block partials in block order, so results are
// bit-reproducible.
#include <algorithm>
#include <string>

#include "ops.h"

namespace ovl {
namespace {

template <int P>
__device__ inline size_t cx_offset(int row, int h, int Nh) {
  constexpr int cpb = Prec<P>::cpb;
  const int p = row / 12, c = row % 12;
  const size_t blk = (static_cast<size_t>(p) * (12 / cpb) + c / cpb) * Nh + h;
  return blk * 16 + (c % cpb) * (16 / cpb);
}

template <int P>
__device__ inline Cx<double> load_cx(const char* base, int row, int h, int Nh) {
  Cx<typename Prec<P>::real> v = ScalarIO<P>::load1(base + cx_offset<P>(row, h, Nh));
  return {static_cast<double>(v.re), static_cast<double>(v.im)};
}

// Basis elements are read once per sweep: non-temporal, so the batch's
// blocks (reused across the 24 rows of a site tile) stay in L2.
__device__ inline Cx<double> load_basis(const char* base, int row, int h, int Nh) {
  typedef double f64x2_t __attribute__((ext_vector_type(2)));
  const f64x2_t v = __builtin_nontemporal_load(reinterpret_cast<const f64x2_t*>(base + cx_offset<OVL_F64>(row, h, Nh)));
  return {v.x, v.y};
}

template <int P>
__device__ inline void store_cx(char* base, int row, int h, int Nh, Cx<double> v) {
  using real = typename Prec<P>::real;
  ScalarIO<P>::store1(base + cx_offset<P>(row, h, Nh), Cx<real>{static_cast<real>(v.re), static_cast<real>(v.im)});
}

constexpr int PJ_TILE = 64;     // elements per tile (one per lane)
constexpr int PJ_WAVES = 8;     // waves per block of block_dot
constexpr int PJ_BLOCKS = 512;  // K-split of block_dot

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// partial[(i*G + b)*R + r] = sum over K-block b's tiles of conj(V_i) psi_r.
// blockIdx.x selects a group of PJ_WAVES*IW basis vectors (each wave owns
// IW), blockIdx.y the K-block; the groups of one K-block are neighbours in
// launch order, so they share the batch tiles in cache.  Each tile of the
// batch is staged in LDS (as FP64) once per block.
// EX: the batch has exactly RMAX vectors (R is a compile-time constant, so
// per-rhs guards and coefficient strides fold away).
template <int PP, int RMAX, int IW, bool EX>
__global__ __launch_bounds__(PJ_WAVES * 64) void dot_kernel(int Nh, int ell, const char* V, size_t vstrideV,
                                                             const char* psi, size_t vstrideP, int R,
                                                             double2* partial) {
  if constexpr (EX) R = RMAX;
  __shared__ Cx<double> tile[RMAX][PJ_TILE];
  const int tiles_per_row = (Nh + PJ_TILE - 1) / PJ_TILE;
  const long total = 24L * tiles_per_row;
  const int G = gridDim.y, kb = blockIdx.y;
  const long t0 = total * kb / G, t1 = total * (kb + 1) / G;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ibase = (blockIdx.x * PJ_WAVES + wave) * IW;
  Cx<double> acc[IW][RMAX];
#pragma unroll
  for (int j = 0; j < IW; ++j)
#pragma unroll
    for (int r = 0; r < RMAX; ++r) acc[j][r] = {0.0, 0.0};

  // t runs over (tile, row) with the row fastest, so the 24 rows of a site
  // tile, which share the batch's 16-byte blocks, are read back to back
  for (long t = t0; t < t1; ++t) {
    const int row = static_cast<int>(t % 24);
    const int h0 = static_cast<int>(t / 24) * PJ_TILE;
    const int h = h0 + lane;
    // this tile's basis elements are loaded before the barrier
    Cx<double> v[IW];
#pragma unroll
    for (int j = 0; j < IW; ++j)
      v[j] = (ibase + j < ell && h < Nh) ? load_basis(V + (ibase + j) * vstrideV, row, h, Nh)
                                         : Cx<double>{0.0, 0.0};
    __syncthreads();
    for (int k = threadIdx.x; k < R * PJ_TILE; k += blockDim.x) {
      const int r = k / PJ_TILE, l = k % PJ_TILE;
      tile[r][l] = (h0 + l < Nh) ? load_cx<PP>(psi + r * vstrideP, row, h0 + l, Nh) : Cx<double>{0.0, 0.0};
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      const Cx<double> ps = (r < R) ? tile[r][lane] : Cx<double>{0.0, 0.0};
#pragma unroll
      for (int j = 0; j < IW; ++j) {  // acc += conj(v) ps, four FMAs
        acc[j][r].re = fma(v[j].re, ps.re, acc[j][r].re);
        acc[j][r].re = fma(v[j].im, ps.im, acc[j][r].re);
        acc[j][r].im = fma(v[j].re, ps.im, acc[j][r].im);
        acc[j][r].im = fma(-v[j].im, ps.re, acc[j][r].im);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < IW; ++j) {
    const int i = ibase + j;
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      const double re = wsum(acc[j][r].re), im = wsum(acc[j][r].im);
      if (lane == 0 && i < ell && r < R)
        partial[(static_cast<size_t>(i) * G + kb) * R + r] = make_double2(re, im);
    }
  }
}

// C[i*R + r] = sum_b partial[(i*G + b)*R + r], in block order.
__global__ void dot_reduce_kernel(int ell, int R, int G, const double2* partial, double2* C) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ell * R) return;
  const int i = k / R, r = k % R;
  double re = 0.0, im = 0.0;
  for (int b = 0; b < G; ++b) {
    const double2 v = partial[(static_cast<size_t>(i) * G + b) * R + r];
    re += v.x;
    im += v.y;
  }
  C[k] = make_double2(re, im);
}

// Y_r = [Y_r] + sum_i V_i K[i*R + r]; one thread per element, K in LDS.
template <int PP, int RMAX, bool KEEP, bool EX>
__global__ __launch_bounds__(256) void axpy_kernel(int Nh, int ell, const char* V, size_t vstrideV,
                                                   const double2* __restrict__ coef, char* Y, size_t vstrideP,
                                                   int R) {
  if constexpr (EX) R = RMAX;
  // coef[i*R + r] is the same for the whole wave: scalar loads
  const int row = blockIdx.x % 24;  // rows of a site tile in consecutive blocks
  const int h = (blockIdx.x / 24) * blockDim.x + threadIdx.x;
  if (h >= Nh) return;
  Cx<double> y[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r)
    y[r] = (KEEP && r < R) ? load_cx<PP>(Y + r * vstrideP, row, h, Nh) : Cx<double>{0.0, 0.0};
  for (int i = 0; i < ell; ++i) {
    const Cx<double> v = load_basis(V + i * vstrideV, row, h, Nh);
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      if (r < R) {
        const double2 cc = coef[i * R + r];
        y[r].re = fma(v.re, cc.x, y[r].re);
        y[r].re = fma(-v.im, cc.y, y[r].re);
        y[r].im = fma(v.re, cc.y, y[r].im);
        y[r].im = fma(v.im, cc.x, y[r].im);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RMAX; ++r)
    if (r < R) store_cx<PP>(Y + r * vstrideP, row, h, Nh, y[r]);
}

// psi_h = psi - sum_i C_i eta_i, w = [gamma5] sum_i sign_i C_i eta_i.
template <int PP, int RMAX, bool EX>
__global__ __launch_bounds__(256) void project_kernel(int Nh, int ell, const char* V, size_t vstrideV,
                                                      const char* psi, char* psih, char* w, size_t vstrideP, int R,
                                                      const double2* __restrict__ coef,
                                                      const double* __restrict__ sgn, int g5w) {
  if constexpr (EX) R = RMAX;
  // coef[i*R + r] and sgn[i] are the same for the whole wave: scalar loads
  const int row = blockIdx.x % 24;  // rows of a site tile in consecutive blocks
  const int h = (blockIdx.x / 24) * blockDim.x + threadIdx.x;
  if (h >= Nh) return;
  Cx<double> ph[RMAX], ww[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    ph[r] = (r < R) ? load_cx<PP>(psi + r * vstrideP, row, h, Nh) : Cx<double>{0.0, 0.0};
    ww[r] = {0.0, 0.0};
  }
  // the basis elements of the next PF modes are in flight while one is used
  constexpr int PF = 4;
  Cx<double> vb[PF];
#pragma unroll
  for (int k = 0; k < PF; ++k) vb[k] = (k < ell) ? load_basis(V + k * vstrideV, row, h, Nh) : Cx<double>{0.0, 0.0};
  for (int i0 = 0; i0 < ell; i0 += PF) {
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int i = i0 + k;
      if (i < ell) {
        const Cx<double> v = vb[k];
        if (i + PF < ell) vb[k] = load_basis(V + (i + PF) * vstrideV, row, h, Nh);
        const double s = sgn[i];
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
          if (r < R) {
            const double2 cc = coef[i * R + r];
            const double vr = v.re * cc.x - v.im * cc.y, vi = v.re * cc.y + v.im * cc.x;
            ph[r].re -= vr;
            ph[r].im -= vi;
            ww[r].re = fma(s, vr, ww[r].re);
            ww[r].im = fma(s, vi, ww[r].im);
          }
        }
      }
    }
  }
  const double gs = (g5w && (row % 12) >= 6) ? -1.0 : 1.0;  // spins 2, 3 under gamma5
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    if (r < R) {
      store_cx<PP>(psih + r * vstrideP, row, h, Nh, ph[r]);
      store_cx<PP>(w + r * vstrideP, row, h, Nh, gs * ww[r]);
    }
  }
}

// In-place basis rotation V[:, j] = sum_{i<K} V[:, i] S[i + K j], j < k.
// Each block stages all K values of RT consecutive elements of one row in
// LDS, so every element is read once and rewritten by the same block.
constexpr int RT = 8;
__global__ __launch_bounds__(256) void rotate_kernel(int Nh, int K, int k, char* V, size_t vstride,
                                                     const double2* S) {
  extern __shared__ Cx<double> vt[];  // [K][RT]
  const int row = blockIdx.y;
  const int h0 = blockIdx.x * RT;
  for (int idx = threadIdx.x; idx < K * RT; idx += blockDim.x) {
    const int i = idx / RT, e = idx % RT;
    vt[idx] = (h0 + e < Nh) ? load_cx<OVL_F64>(V + i * vstride, row, h0 + e, Nh) : Cx<double>{0.0, 0.0};
  }
  __syncthreads();
  const int e = threadIdx.x % RT;
  for (int j = threadIdx.x / RT; j < k; j += blockDim.x / RT) {
    Cx<double> acc = {0.0, 0.0};
    const double2* sj = S + static_cast<size_t>(K) * j;
    for (int i = 0; i < K; ++i) {
      const double2 c = sj[i];
      acc = acc + vt[i * RT + e] * Cx<double>{c.x, c.y};
    }
    if (h0 + e < Nh) store_cx<OVL_F64>(V + j * vstride, row, h0 + e, Nh, acc);
  }
}

template <int PP, int RMAX, int IW, bool EX = false>
void dot_go(const ovl_geom* g, const void* V, int ell, const void* psi, int R, double2* C, double2* part, int G,
            hipStream_t s) {
  const int Nh = g->geo.Nh;
  const size_t vsV = spinor_vec_bytes(g, OVL_F64), vsP = spinor_vec_bytes(g, PP);
  const int groups = (ell + PJ_WAVES * IW - 1) / (PJ_WAVES * IW);
  hipLaunchKernelGGL((dot_kernel<PP, RMAX, IW, EX>), dim3(groups, G), dim3(PJ_WAVES * 64), 0, s, Nh, ell,
                     static_cast<const char*>(V), vsV, static_cast<const char*>(psi), vsP, R, part);
  OVL_HIP(hipGetLastError());
  hipLaunchKernelGGL(dot_reduce_kernel, dim3((ell * R + 255) / 256), dim3(256), 0, s, ell, R, G,
                     static_cast<const double2*>(part), C);
  OVL_HIP(hipGetLastError());
}

// C = V^dag psi with the per-block partials in `part` (ell * G * R entries).
template <int PP>
void dot_r(const ovl_geom* g, const void* V, int ell, const void* psi, int R, double2* C, double2* part, int G,
           hipStream_t s) {
  if (R == 1) dot_go<PP, 1, 8, true>(g, V, ell, psi, R, C, part, G, s);
  else if (R <= 4) dot_go<PP, 4, 4>(g, V, ell, psi, R, C, part, G, s);
  else if (R == 12) dot_go<PP, 12, 2, true>(g, V, ell, psi, R, C, part, G, s);
  else dot_go<PP, 12, 2>(g, V, ell, psi, R, C, part, G, s);
}

void dot_prec(const ovl_geom* g, const void* V, int ell, const void* psi, int prec, int R, double2* C, double2* part,
              int G, hipStream_t s) {
  switch (prec) {
    case OVL_F64: dot_r<OVL_F64>(g, V, ell, psi, R, C, part, G, s); break;
    case OVL_F32: dot_r<OVL_F32>(g, V, ell, psi, R, C, part, G, s); break;
    case OVL_F16: dot_r<OVL_F16>(g, V, ell, psi, R, C, part, G, s); break;
    case OVL_BF16: dot_r<OVL_BF16>(g, V, ell, psi, R, C, part, G, s); break;
    default: throw Error(OVL_E_PRECISION, "unknown precision");
  }
}

template <int PP, int RMAX, bool EX = false>
void axpy_go(const ovl_geom* g, const void* V, int ell, const double2* K, void* Y, int R, bool keep, hipStream_t s) {
  const int Nh = g->geo.Nh;
  const size_t vsV = spinor_vec_bytes(g, OVL_F64), vsP = spinor_vec_bytes(g, PP);
  dim3 grid(((Nh + 255) / 256) * 24);
  if (keep)
    hipLaunchKernelGGL((axpy_kernel<PP, RMAX, true, EX>), grid, dim3(256), 0, s, Nh, ell, static_cast<const char*>(V),
                       vsV, K, static_cast<char*>(Y), vsP, R);
  else
    hipLaunchKernelGGL((axpy_kernel<PP, RMAX, false, EX>), grid, dim3(256), 0, s, Nh, ell,
                       static_cast<const char*>(V), vsV, K, static_cast<char*>(Y), vsP, R);
  OVL_HIP(hipGetLastError());
}

template <int PP>
void axpy_r(const ovl_geom* g, const void* V, int ell, const double2* K, void* Y, int R, bool keep, hipStream_t s) {
  if (R == 1) axpy_go<PP, 1, true>(g, V, ell, K, Y, R, keep, s);
  else if (R <= 4) axpy_go<PP, 4>(g, V, ell, K, Y, R, keep, s);
  else if (R == 12) axpy_go<PP, 12, true>(g, V, ell, K, Y, R, keep, s);
  else axpy_go<PP, 12>(g, V, ell, K, Y, R, keep, s);
}

template <int PP, int RMAX, bool EX = false>
void project_go(const ovl_lowmodes* lm, const void* psi, void* psih, void* w, int R, int g5w, const double2* C,
                hipStream_t s) {
  const ovl_geom* g = &lm->geom;
  const int Nh = g->geo.Nh;
  const size_t vsV = spinor_vec_bytes(g, OVL_F64), vsP = spinor_vec_bytes(g, PP);
  hipLaunchKernelGGL((project_kernel<PP, RMAX, EX>), dim3(((Nh + 255) / 256) * 24), dim3(256), 0, s, Nh, lm->ell,
                     static_cast<const char*>(lm->V), vsV, static_cast<const char*>(psi), static_cast<char*>(psih),
                     static_cast<char*>(w), vsP, R, C, lm->dev_sign, g5w);
  OVL_HIP(hipGetLastError());
}

template <int PP>
void project_r(const ovl_lowmodes* lm, const void* psi, void* psih, void* w, int R, int g5w, const double2* C,
               hipStream_t s) {
  if (R == 1) project_go<PP, 1, true>(lm, psi, psih, w, R, g5w, C, s);
  else if (R <= 4) project_go<PP, 4>(lm, psi, psih, w, R, g5w, C, s);
  else if (R == 12) project_go<PP, 12, true>(lm, psi, psih, w, R, g5w, C, s);
  else project_go<PP, 12>(lm, psi, psih, w, R, g5w, C, s);
}

}  // namespace

void block_dot(const ovl_geom* g, const void* V, int ell, const void* psi, int prec, int R, double2* C,
               hipStream_t s) {
  OVL_REQUIRE(R >= 1 && R <= OVL_MAX_RHS && ell >= 1, OVL_E_ARG, "block_dot: 1 <= R <= 12, ell >= 1");
  WsBuf part(static_cast<size_t>(ell) * PJ_BLOCKS * R * sizeof(double2), s);
  dot_prec(g, V, ell, psi, prec, R, C, static_cast<double2*>(part.p), PJ_BLOCKS, s);
}

void block_axpy(const ovl_geom* g, const void* V, int ell, const double2* K, void* Y, int prec, int R, bool keep,
                hipStream_t s) {
  OVL_REQUIRE(R >= 1 && R <= OVL_MAX_RHS && ell >= 1, OVL_E_ARG, "block_axpy: 1 <= R <= 12, ell >= 1");
  switch (prec) {
    case OVL_F64: axpy_r<OVL_F64>(g, V, ell, K, Y, R, keep, s); break;
    case OVL_F32: axpy_r<OVL_F32>(g, V, ell, K, Y, R, keep, s); break;
    case OVL_F16: axpy_r<OVL_F16>(g, V, ell, K, Y, R, keep, s); break;
    case OVL_BF16: axpy_r<OVL_BF16>(g, V, ell, K, Y, R, keep, s); break;
    default: throw Error(OVL_E_PRECISION, "unknown precision");
  }
}

void block_rotate_inplace(const ovl_geom* g, void* V, int K, const double2* S, int k, hipStream_t s) {
  OVL_REQUIRE(k >= 1 && k <= K, OVL_E_ARG, "rotate: need 1 <= k <= K");
  const size_t lds = static_cast<size_t>(K) * RT * sizeof(Cx<double>);
  OVL_REQUIRE(lds <= 64 * 1024, OVL_E_ARG, "rotate: basis too large (K <= 512)");
  const int Nh = g->geo.Nh;
  dim3 grid((Nh + RT - 1) / RT, 24);
  hipLaunchKernelGGL(rotate_kernel, grid, dim3(256), lds, s, Nh, K, k, static_cast<char*>(V),
                     spinor_vec_bytes(g, OVL_F64), S);
  OVL_HIP(hipGetLastError());
}

namespace {
// The projection with caller-provided scratch: C (ell * nrhs coefficients)
// and the split-K partials of pass 1 (ell * G * nrhs).
void lowmode_project_ws(const ovl_lowmodes* lm, const void* psi, void* psih, void* w, int prec, int nrhs, int g5w,
                        double2* C, double2* part, int G, hipStream_t s) {
  OVL_REQUIRE(nrhs >= 1 && nrhs <= OVL_MAX_RHS && lm->ell >= 1, OVL_E_ARG,
              "projection: 1 <= nrhs <= 12 and at least one low mode");
  dot_prec(&lm->geom, lm->V, lm->ell, psi, prec, nrhs, C, part, G, s);
  switch (prec) {
    case OVL_F64: project_r<OVL_F64>(lm, psi, psih, w, nrhs, g5w, C, s); break;
    case OVL_F32: project_r<OVL_F32>(lm, psi, psih, w, nrhs, g5w, C, s); break;
    case OVL_F16: project_r<OVL_F16>(lm, psi, psih, w, nrhs, g5w, C, s); break;
    case OVL_BF16: project_r<OVL_BF16>(lm, psi, psih, w, nrhs, g5w, C, s); break;
    default: throw Error(OVL_E_PRECISION, "unknown precision");
  }
}

// Scratch of the allocation-free projection: one array per GPU, in device
// memory for the life of the process.  Host code never uses the array's
// name as an address; the kernels receive the per-device pointer that
// hipGetSymbolAddress returns.
constexpr size_t kStaticScratchBytes = size_t(16) << 20;
constexpr int kStaticMinBlocks = 64;  // fewest K-blocks of pass 1 accepted
// Largest ell * nrhs for which the coefficients (rounded up to 256 bytes)
// and kStaticMinBlocks sets of partials fit.
constexpr size_t kMaxStaticEllRhs = (kStaticScratchBytes - 256) / (sizeof(double2) * (kStaticMinBlocks + 1));
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
void* static_scratch() {
  int dev = -1;
  OVL_HIP(hipGetDevice(&dev));
  OVL_REQUIRE(dev >= 0 && dev < kMaxDevices, OVL_E_ARG, "device index out of range for the static scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      throw Error(OVL_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

void lowmode_project(const ovl_lowmodes* lm, const void* psi, void* psih, void* w, int prec, int nrhs, int g5w,
                     hipStream_t s) {
  OVL_REQUIRE(nrhs >= 1 && nrhs <= OVL_MAX_RHS, OVL_E_ARG, "projection supports 1 to 12 right-hand sides");
  WsBuf cbuf(static_cast<size_t>(lm->ell) * nrhs * sizeof(double2), s);
  WsBuf part(static_cast<size_t>(lm->ell) * PJ_BLOCKS * nrhs * sizeof(double2), s);
  lowmode_project_ws(lm, psi, psih, w, prec, nrhs, g5w, static_cast<double2*>(cbuf.p),
                     static_cast<double2*>(part.p), PJ_BLOCKS, s);
}

// Same projection with its scratch in the static per-device array.  Pass 1
// keeps PJ_BLOCKS K-blocks while they fit (then the result is bit-identical
// to lowmode_project), else as many as fit, at least kStaticMinBlocks.
// Every partial and coefficient slot is written before it is read, so
// nothing needs clearing between calls.
void lowmode_project_static(const ovl_lowmodes* lm, const void* psi, void* psih, void* w, int prec, int nrhs,
                            hipStream_t s) {
  OVL_REQUIRE(nrhs >= 1 && nrhs <= OVL_MAX_RHS, OVL_E_ARG, "projection supports 1 to 12 right-hand sides");
  OVL_REQUIRE(static_cast<size_t>(lm->ell) * nrhs <= kMaxStaticEllRhs, OVL_E_ARG,
              "ovl_lowmodes_project_noalloc: ell * nrhs = " + std::to_string(lm->ell * nrhs) +
                  " exceeds what its 16 MiB static scratch holds (ell * nrhs <= " +
                  std::to_string(kMaxStaticEllRhs) + ")");
  const size_t unit = static_cast<size_t>(lm->ell) * nrhs * sizeof(double2);  // one coefficient set
  const size_t c_bytes = (unit + 255) / 256 * 256;
  const size_t fit = (kStaticScratchBytes - c_bytes) / unit;  // >= kStaticMinBlocks by the check above
  const int G = static_cast<int>(std::min<size_t>(PJ_BLOCKS, fit));
  char* base = static_cast<char*>(static_scratch());
  lowmode_project_ws(lm, psi, psih, w, prec, nrhs, 0, reinterpret_cast<double2*>(base),
                     reinterpret_cast<double2*>(base + c_bytes), G, s);
}

}  // namespace ovl
