// Lattice geometry, spinor packing and gauge-link packing.
//
// Site order (Sec. II, Fig. 1; the layout itself is this library's choice):
// lex = x + Lx*(y + Ly*(z + Lz*t)), parity p = (x+y+z+t) mod 2, even-odd
// index eo = p*N/2 + lex/2.  Device fields are structure-of-arrays over the
// N/2 sites of each parity (see ovl.h).
#include <cmath>

#include "ops.h"

namespace ovl {
namespace {

__device__ inline int lex_of(const Geo& g, int x, int y, int z, int t) {
  return x + g.Lx * (y + g.Ly * (z + g.Lz * t));
}

__global__ void neighbor_table_kernel(Geo g, int32_t* table) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = 2 * g.Nh;
  if (e >= N) return;
  const int p = e >= g.Nh;
  const int h = e - p * g.Nh;
  int x, y, z, t, nb[8];
  site_coords(g, p, h, x, y, z, t);
  site_neighbors(g, h, x, y, z, t, nb);
  for (int d = 0; d < 8; ++d) table[static_cast<size_t>(d) * N + e] = (1 - p) * g.Nh + nb[d];
}

// AoS complex128 [rhs][N lex][12] <-> library layout, one thread per eo site.
template <int P>
__global__ void pack_kernel(Geo g, const double2* aos, void* out, size_t vbytes) {
  using real = typename Prec<P>::real;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * g.Nh) return;
  const int p = e >= g.Nh, h = e - p * g.Nh;
  int x, y, z, t;
  site_coords(g, p, h, x, y, z, t);
  const size_t src = (static_cast<size_t>(blockIdx.y) * 2 * g.Nh + lex_of(g, x, y, z, t)) * 12;
  Cx<real> s[12];
  for (int c = 0; c < 12; ++c) {
    double2 v = aos[src + c];
    s[c] = {static_cast<real>(v.x), static_cast<real>(v.y)};
  }
  SpinorIO<P>::store(static_cast<char*>(out) + blockIdx.y * vbytes, p, h, g.Nh, s);
}

template <int P>
__global__ void unpack_kernel(Geo g, const void* in, double2* aos, size_t vbytes) {
  using real = typename Prec<P>::real;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * g.Nh) return;
  const int p = e >= g.Nh, h = e - p * g.Nh;
  int x, y, z, t;
  site_coords(g, p, h, x, y, z, t);
  Cx<real> s[12];
  SpinorIO<P>::load(static_cast<const char*>(in) + blockIdx.y * vbytes, p, h, g.Nh, s);
  const size_t dst = (static_cast<size_t>(blockIdx.y) * 2 * g.Nh + lex_of(g, x, y, z, t)) * 12;
  for (int c = 0; c < 12; ++c) aos[dst + c] = make_double2(static_cast<double>(s[c].re), static_cast<double>(s[c].im));
}

template <int P, int R>
__global__ void gauge_pack_kernel(Geo g, const double2* aos, void* links) {
  using F = LinkFmt<P, R>;
  using real = typename Prec<P>::real;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * g.Nh) return;
  const int p = e >= g.Nh, h = e - p * g.Nh;
  int x, y, z, t;
  site_coords(g, p, h, x, y, z, t);
  const size_t src = static_cast<size_t>(lex_of(g, x, y, z, t)) * 36;
  for (int mu = 0; mu < 4; ++mu) {
    char* b = static_cast<char*>(links) + ((static_cast<size_t>(mu) * 2 + p) * F::K * g.Nh + h) * F::E;
    Cx<real> c[9];
    for (int k = 0; k < 9; ++k) {
      double2 v = aos[src + mu * 9 + k];
      c[k] = {static_cast<real>(v.x), static_cast<real>(v.y)};
    }
    if constexpr (F::cpe == 1) {
      for (int k = 0; k < F::ncx; ++k) ScalarIO<P>::store1(b + static_cast<size_t>(k) * g.Nh * F::E, c[k]);
    } else {
      for (int k = 0; k < F::K; ++k) ScalarIO<P>::store2(b + static_cast<size_t>(k) * g.Nh * F::E, c + 2 * k);
    }
  }
}

// Rebuild representation (P, R) from the FP64 18-real master copy.
template <int P, int R>
__global__ void gauge_repack_kernel(Geo g, const void* master, void* links) {
  using F = LinkFmt<P, R>;
  using real = typename Prec<P>::real;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * g.Nh) return;
  const int p = e >= g.Nh, h = e - p * g.Nh;
  for (int mu = 0; mu < 4; ++mu) {
    Cx<double> u[3][3];
    LinkIO<OVL_F64, 18>::load(master, mu, p, h, g.Nh, u);
    Cx<real> c[9];
    for (int k = 0; k < 9; ++k) c[k] = {static_cast<real>(u[k / 3][k % 3].re), static_cast<real>(u[k / 3][k % 3].im)};
    char* b = static_cast<char*>(links) + ((static_cast<size_t>(mu) * 2 + p) * F::K * g.Nh + h) * F::E;
    if constexpr (F::cpe == 1) {
      for (int k = 0; k < F::ncx; ++k) ScalarIO<P>::store1(b + static_cast<size_t>(k) * g.Nh * F::E, c[k]);
    } else {
      for (int k = 0; k < F::K; ++k) ScalarIO<P>::store2(b + static_cast<size_t>(k) * g.Nh * F::E, c + 2 * k);
    }
  }
}

// Per block: max over links of max(|U^dag U - 1|_max, |det U - 1|), read
// from the FP64 master.  NaN counts as +inf.
__global__ void su3_deviation_kernel(Geo g, const void* master, double* block_max) {
  __shared__ double red[256];
  double dev = 0.0;
  const int64_t nlinks = static_cast<int64_t>(8) * g.Nh;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < nlinks;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int h = static_cast<int>(i % g.Nh);
    const int mp = static_cast<int>(i / g.Nh);  // mu*2 + p
    Cx<double> u[3][3];
    LinkIO<OVL_F64, 18>::load(master, mp >> 1, mp & 1, h, g.Nh, u);
    double d = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        Cx<double> s = {0.0, 0.0};
        for (int c = 0; c < 3; ++c) s = s + cmul_conj(u[c][a], u[c][b]);
        s.re -= (a == b) ? 1.0 : 0.0;
        d = fmax(d, fmax(fabs(s.re), fabs(s.im)));
      }
    Cx<double> det = u[0][0] * (u[1][1] * u[2][2] - u[1][2] * u[2][1]) -
                     u[0][1] * (u[1][0] * u[2][2] - u[1][2] * u[2][0]) +
                     u[0][2] * (u[1][0] * u[2][1] - u[1][1] * u[2][0]);
    d = fmax(d, hypot(det.re - 1.0, det.im));
    if (!(d == d)) d = INFINITY;
    dev = fmax(dev, d);
  }
  red[threadIdx.x] = dev;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) block_max[blockIdx.x] = red[0];
}

template <int P, int R>
void gauge_pack(const Geo& g, const double2* aos, void* links, hipStream_t s) {
  const int N = 2 * g.Nh;
  hipLaunchKernelGGL((gauge_pack_kernel<P, R>), dim3((N + 255) / 256), dim3(256), 0, s, g, aos, links);
  OVL_HIP(hipGetLastError());
}

size_t link_bytes(const ovl_geom* g, int prec, int recon) {
  size_t per = 0;
  if (prec == OVL_F64) per = recon * 8;
  else if (prec == OVL_F32) per = recon * 4;
  else per = recon * 2;
  return per * 4 * static_cast<size_t>(g->N);
}

}  // namespace

void check_prec(int prec) {
  OVL_REQUIRE(prec >= OVL_F64 && prec <= OVL_BF16, OVL_E_PRECISION, "unknown precision");
}
void check_nrhs(int nrhs) {
  OVL_REQUIRE(nrhs >= 1 && nrhs <= 4096, OVL_E_ARG, "nrhs out of range");
}

Geo make_geo(const int* d) {
  Geo g;
  g.Lx = d[0];
  g.Ly = d[1];
  g.Lz = d[2];
  g.Lt = d[3];
  g.lxh = d[0] / 2;
  g.sy = g.lxh;
  g.sz = g.lxh * d[1];
  g.st = g.lxh * d[1] * d[2];
  g.Nh = g.st * d[3];
  return g;
}

void neighbor_table(const ovl_geom* g, int32_t* dev, hipStream_t s) {
  const int N = static_cast<int>(g->N);
  hipLaunchKernelGGL(neighbor_table_kernel, dim3((N + 255) / 256), dim3(256), 0, s, g->geo, dev);
  OVL_HIP(hipGetLastError());
}

void pack_spinor(const ovl_geom* g, const double* aos, void* out, int prec, int nrhs, hipStream_t s) {
  const int N = static_cast<int>(g->N);
  dim3 grid((N + 255) / 256, nrhs);
  const size_t vb = spinor_vec_bytes(g, prec);
  const double2* a = reinterpret_cast<const double2*>(aos);
  switch (prec) {
    case OVL_F64: hipLaunchKernelGGL(pack_kernel<OVL_F64>, grid, dim3(256), 0, s, g->geo, a, out, vb); break;
    case OVL_F32: hipLaunchKernelGGL(pack_kernel<OVL_F32>, grid, dim3(256), 0, s, g->geo, a, out, vb); break;
    case OVL_F16: hipLaunchKernelGGL(pack_kernel<OVL_F16>, grid, dim3(256), 0, s, g->geo, a, out, vb); break;
    case OVL_BF16: hipLaunchKernelGGL(pack_kernel<OVL_BF16>, grid, dim3(256), 0, s, g->geo, a, out, vb); break;
  }
  OVL_HIP(hipGetLastError());
}

void unpack_spinor(const ovl_geom* g, const void* in, double* aos, int prec, int nrhs, hipStream_t s) {
  const int N = static_cast<int>(g->N);
  dim3 grid((N + 255) / 256, nrhs);
  const size_t vb = spinor_vec_bytes(g, prec);
  double2* a = reinterpret_cast<double2*>(aos);
  switch (prec) {
    case OVL_F64: hipLaunchKernelGGL(unpack_kernel<OVL_F64>, grid, dim3(256), 0, s, g->geo, in, a, vb); break;
    case OVL_F32: hipLaunchKernelGGL(unpack_kernel<OVL_F32>, grid, dim3(256), 0, s, g->geo, in, a, vb); break;
    case OVL_F16: hipLaunchKernelGGL(unpack_kernel<OVL_F16>, grid, dim3(256), 0, s, g->geo, in, a, vb); break;
    case OVL_BF16: hipLaunchKernelGGL(unpack_kernel<OVL_BF16>, grid, dim3(256), 0, s, g->geo, in, a, vb); break;
  }
  OVL_HIP(hipGetLastError());
}

double su3_deviation(const ovl_gauge* u, hipStream_t s) {
  constexpr int NB = 1024;
  WsBuf buf(NB * sizeof(double), s);
  hipLaunchKernelGGL(su3_deviation_kernel, dim3(NB), dim3(256), 0, s, u->geom.geo, u->master,
                     static_cast<double*>(buf.p));
  OVL_HIP(hipGetLastError());
  std::vector<double> host(NB);
  OVL_HIP(hipMemcpyAsync(host.data(), buf.p, NB * sizeof(double), hipMemcpyDeviceToHost, s));
  OVL_HIP(hipStreamSynchronize(s));
  double m = 0.0;
  for (double v : host) m = (v > m || v != v) ? v : m;
  return m;
}

void gauge_create_master(ovl_gauge* u, const double* aos, hipStream_t s) {
  const ovl_geom* g = &u->geom;
  OVL_HIP(hipMalloc(&u->master, link_bytes(g, OVL_F64, 18)));
  mem_track(static_cast<int64_t>(link_bytes(g, OVL_F64, 18)));
  gauge_pack<OVL_F64, 18>(g->geo, reinterpret_cast<const double2*>(aos), u->master, s);
  OVL_HIP(hipStreamSynchronize(s));
  u->links[OVL_F64] = u->master;
  u->recon[OVL_F64] = 18;
}

template <int P, int R>
void repack(const Geo& g, const void* master, void* dst, hipStream_t s) {
  const int N = 2 * g.Nh;
  hipLaunchKernelGGL((gauge_repack_kernel<P, R>), dim3((N + 255) / 256), dim3(256), 0, s, g, master, dst);
  OVL_HIP(hipGetLastError());
}

void gauge_set_repr(ovl_gauge* u, int prec, int recon, hipStream_t s) {
  const ovl_geom* g = &u->geom;
  if (prec == OVL_F64 && recon == 18) {
    if (u->links[OVL_F64] && u->links[OVL_F64] != u->master) {
      OVL_HIP(hipFree(u->links[OVL_F64]));
      mem_track(-static_cast<int64_t>(link_bytes(g, OVL_F64, u->recon[OVL_F64])));
    }
    u->links[OVL_F64] = u->master;
    u->recon[OVL_F64] = 18;
    return;
  }
  void* dst = nullptr;
  OVL_HIP(hipMalloc(&dst, link_bytes(g, prec, recon)));
  mem_track(static_cast<int64_t>(link_bytes(g, prec, recon)));
  try {
    const bool r18 = recon == 18;
    switch (prec) {
      case OVL_F64: repack<OVL_F64, 12>(g->geo, u->master, dst, s); break;
      case OVL_F32: r18 ? repack<OVL_F32, 18>(g->geo, u->master, dst, s) : repack<OVL_F32, 12>(g->geo, u->master, dst, s); break;
      case OVL_F16: r18 ? repack<OVL_F16, 18>(g->geo, u->master, dst, s) : repack<OVL_F16, 12>(g->geo, u->master, dst, s); break;
      case OVL_BF16: r18 ? repack<OVL_BF16, 18>(g->geo, u->master, dst, s) : repack<OVL_BF16, 12>(g->geo, u->master, dst, s); break;
    }
    OVL_HIP(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipFree(dst);
    mem_track(-static_cast<int64_t>(link_bytes(g, prec, recon)));
    throw;
  }
  if (u->links[prec] && u->links[prec] != u->master) {
    OVL_HIP(hipFree(u->links[prec]));
    mem_track(-static_cast<int64_t>(link_bytes(g, prec, u->recon[prec])));
  }
  u->links[prec] = dst;
  u->recon[prec] = recon;
}

void gauge_free(ovl_gauge* u) {
  const ovl_geom* g = &u->geom;
  for (int p = 0; p < 4; ++p)
    if (u->links[p] && u->links[p] != u->master) {
      (void)hipFree(u->links[p]);
      mem_track(-static_cast<int64_t>(link_bytes(g, p, u->recon[p])));
    }
  if (u->master) {
    (void)hipFree(u->master);
    mem_track(-static_cast<int64_t>(link_bytes(g, OVL_F64, 18)));
  }
}

const void* gauge_links(const ovl_gauge* u, int prec, int* recon) {
  OVL_REQUIRE(u->links[prec] != nullptr, OVL_E_PRECISION,
              "no link representation for this precision (call ovl_gauge_set_repr)");
  *recon = u->recon[prec];
  return u->links[prec];
}

}  // namespace ovl
