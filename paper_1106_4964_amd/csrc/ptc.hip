// Gauge-equivariant parallel-transport convolution (PTC) network used as a
// learned right preconditioner for D(m).  Not part of arXiv:1106.4964; it
// is built from the same parallel transporters T_mu as the Wilson operator
// (Sec. II eq. 2, here without the spin projector):
//
//   phi_out[a](x) = sum_b sum_k W[k][a][b] (T_k phi_in[b])(x),
//   k = 0: identity; 1..4: T_{+mu} phi(x) = U_mu(x) phi(x+mu);
//   5..8: T_{-mu} phi(x) = U_mu(x-mu)^dag phi(x-mu);  W[k][a][b]: 4x4 on spin.
//
// Layers are linear, so the network commutes with gauge transformations.
// With T_{+mu}^dag = T_{-mu} and W acting on spin only, the input gradient
// of a layer is the same kind of layer with weights W'[k'][b][a] =
// W[k][a][b]^dag (k' the opposite path), so one forward kernel serves both
// directions.  The weight gradient
//   G[k][a][b] = sum_x sum_colour g_out[a](x) (T_k phi_in[b](x))^dag
// is a site reduction (FP32 per thread, FP64 across blocks, fixed order).
//
// Activations are FP32 spinors in the library layout, one vector per
// channel; the links come from the FP32 representation of the gauge field.
#include <cmath>
#include <complex>

#include "ops.h"

namespace ovl {
namespace {

constexpr int NPATH = 9;
constexpr int CMAX = 4;

// T_k psi at site (p, h) for a FP32 spinor field (k in 0..8).
template <int R>
__device__ inline void transport(const Geo& g, const void* links, const char* f, int p, int h, const int* nb, int k,
                                 Cx<float>* out) {
  if (k == 0) {
    SpinorIO<OVL_F32>::load(f, p, h, g.Nh, out);
    return;
  }
  const int q = 1 - p;
  Cx<float> s[12], u[3][3];
  if (k <= 4) {
    const int mu = k - 1;
    SpinorIO<OVL_F32>::load(f, q, nb[mu], g.Nh, s);
    LinkIO<OVL_F32, R>::load(links, mu, p, h, g.Nh, u);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        Cx<float> r = {0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 3; ++b) r = r + u[a][b] * s[3 * sp + b];
        out[3 * sp + a] = r;
      }
  } else {
    const int mu = k - 5;
    SpinorIO<OVL_F32>::load(f, q, nb[mu + 4], g.Nh, s);
    LinkIO<OVL_F32, R>::load(links, mu, q, nb[mu + 4], g.Nh, u);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        Cx<float> r = {0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 3; ++b) r = r + cmul_conj(u[b][a], s[3 * sp + b]);
        out[3 * sp + a] = r;
      }
  }
}

// out[a] = sum_b sum_k W[k][a][b] T_k in[b]; W in LDS as float2 [k][a][b][s][t].
// blockIdx.y selects one field of a batch: its channels start rstride_in
// (rstride_out) bytes after the previous field's.
template <int R>
__global__ __launch_bounds__(256) void ptc_forward_kernel(Geo g, const void* links, const char* in, char* out,
                                                          size_t vstride, int cin, int cout, const float2* W,
                                                          size_t rstride_in, size_t rstride_out) {
  __shared__ float2 w[NPATH * CMAX * CMAX * 16];
  in += blockIdx.y * rstride_in;
  out += blockIdx.y * rstride_out;
  const int nw = NPATH * cin * cout * 16;
  for (int i = threadIdx.x; i < nw; i += blockDim.x) w[i] = W[i];
  __syncthreads();
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * g.Nh) return;
  const int p = e >= g.Nh, h = e - p * g.Nh;
  int x, y, z, t, nb[8];
  site_coords(g, p, h, x, y, z, t);
  site_neighbors(g, h, x, y, z, t, nb);
  Cx<float> acc[CMAX][12];
#pragma unroll
  for (int a = 0; a < CMAX; ++a)
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[a][c] = {0.f, 0.f};
  for (int b = 0; b < cin; ++b) {
    for (int k = 0; k < NPATH; ++k) {
      Cx<float> v[12];
      transport<R>(g, links, in + b * vstride, p, h, nb, k, v);
#pragma unroll
      for (int a = 0; a < CMAX; ++a) {
        if (a < cout) {
          const float2* wk = w + ((k * cout + a) * cin + b) * 16;
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
              const float2 ww = wk[4 * s + tt];
              const Cx<float> wc = {ww.x, ww.y};
#pragma unroll
              for (int c = 0; c < 3; ++c) acc[a][3 * s + c] = acc[a][3 * s + c] + wc * v[3 * tt + c];
            }
        }
      }
    }
  }
  for (int a = 0; a < cout; ++a) SpinorIO<OVL_F32>::store(out + a * vstride, p, h, g.Nh, acc[a]);
}

// partial[(k*G + block)*cout*cin*16 + ...] = sum over the block's sites of
// g_out[a][s][c] conj(T_k in[b][t][c]).  blockIdx.y = k.
template <int R>
__global__ __launch_bounds__(256) void ptc_wgrad_kernel(Geo g, const void* links, const char* in, const char* gout,
                                                        size_t vstride, int cin, int cout, double2* partial) {
  __shared__ float2 red[256 / 64][CMAX * 16];
  const int k = blockIdx.y;
  const int nout = cin * cout * 16;
  Cx<float> acc[CMAX * 16];  // [a*cin+b][s][t] with cin*cout <= 4
#pragma unroll
  for (int i = 0; i < CMAX * 16; ++i) acc[i] = {0.f, 0.f};
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 2 * g.Nh; e += gridDim.x * blockDim.x) {
    const int p = e >= g.Nh, h = e - p * g.Nh;
    int x, y, z, t, nb[8];
    site_coords(g, p, h, x, y, z, t);
    site_neighbors(g, h, x, y, z, t, nb);
    for (int b = 0; b < cin; ++b) {
      Cx<float> v[12];
      transport<R>(g, links, in + b * vstride, p, h, nb, k, v);
      for (int a = 0; a < cout; ++a) {
        Cx<float> go[12];
        SpinorIO<OVL_F32>::load(gout + a * vstride, p, h, g.Nh, go);
        const int base = (a * cin + b) * 16;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int tt = 0; tt < 4; ++tt) {
            Cx<float> r = acc[base + 4 * s + tt];
#pragma unroll
            for (int c = 0; c < 3; ++c) r = r + cmul_conj(v[3 * tt + c], go[3 * s + c]);
            acc[base + 4 * s + tt] = r;
          }
      }
    }
  }
  // cmul_conj(v, go) = conj(v) * go, i.e. go * conj(v) as required
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i = 0; i < nout; ++i) {
    float re = acc[i].re, im = acc[i].im;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      re += __shfl_xor(re, o, 64);
      im += __shfl_xor(im, o, 64);
    }
    if (lane == 0) red[wv][i] = make_float2(re, im);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nout; i += blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int w = 0; w < 256 / 64; ++w) {
      re += red[w][i].x;
      im += red[w][i].y;
    }
    partial[(static_cast<size_t>(k) * gridDim.x + blockIdx.x) * nout + i] = make_double2(re, im);
  }
}

// out[k][i] (+)= sum_b partial[k][b][i], blocks in order.
__global__ void wgrad_reduce_kernel(int nout, int G, const double2* partial, double2* out, int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= nout) return;
  double re = 0.0, im = 0.0;
  for (int b = 0; b < G; ++b) {
    const double2 v = partial[(static_cast<size_t>(k) * G + b) * nout + i];
    re += v.x;
    im += v.y;
  }
  double2* o = out + static_cast<size_t>(k) * nout + i;
  if (accumulate) {
    re += o->x;
    im += o->y;
  }
  *o = make_double2(re, im);
}

// loss[0] += d2[0] / x2[0];  gscale = (2 / x2[0], 0): the gradient of
// ||out - x||^2 / ||x||^2 with respect to out is gscale * (out - x).
__global__ void pair_loss_kernel(const double* d2, const double* x2, double* loss, double* gscale) {
  if (threadIdx.x == 0) {
    loss[0] += d2[0] / x2[0];
    gscale[0] = 2.0 / x2[0];
    gscale[1] = 0.0;
  }
}

constexpr int WG_BLOCKS = 256;

using zc = std::complex<double>;

// Device copy (float2) of host weights [k][a][b][16].
void upload(const std::vector<zc>& w, float2* dev, hipStream_t s) {
  std::vector<float2> h(w.size());
  for (size_t i = 0; i < w.size(); ++i) h[i] = make_float2(static_cast<float>(w[i].real()), static_cast<float>(w[i].imag()));
  OVL_HIP(hipMemcpyAsync(dev, h.data(), h.size() * sizeof(float2), hipMemcpyHostToDevice, s));
  OVL_HIP(hipStreamSynchronize(s));
}

// W'[k'][b][a] = W[k][a][b]^dag, the weights of the adjoint layer.
std::vector<zc> adjoint_weights(const std::vector<zc>& w, int cin, int cout) {
  std::vector<zc> o(w.size());
  for (int k = 0; k < NPATH; ++k) {
    const int kk = k == 0 ? 0 : (k <= 4 ? k + 4 : k - 4);
    for (int a = 0; a < cout; ++a)
      for (int b = 0; b < cin; ++b)
        for (int s = 0; s < 4; ++s)
          for (int t = 0; t < 4; ++t)
            o[(((kk * cin + b) * cout + a) * 16) + 4 * s + t] = std::conj(w[(((k * cout + a) * cin + b) * 16) + 4 * t + s]);
  }
  return o;
}

struct Layer {
  const ovl_gauge* u;
  const void* links;
  int recon;
  hipStream_t s;
  size_t vstride;

  // nb fields at once: field f reads in + f cin vstride, writes out + f cout vstride
  void forward(const void* in, void* out, int cin, int cout, const float2* W, int nb = 1) const {
    const Geo& g = u->geom.geo;
    dim3 grid((2 * g.Nh + 255) / 256, nb);
    const size_t ri = vstride * cin, ro = vstride * cout;
    if (recon == 18)
      hipLaunchKernelGGL(ptc_forward_kernel<18>, grid, dim3(256), 0, s, g, links, static_cast<const char*>(in),
                         static_cast<char*>(out), vstride, cin, cout, W, ri, ro);
    else
      hipLaunchKernelGGL(ptc_forward_kernel<12>, grid, dim3(256), 0, s, g, links, static_cast<const char*>(in),
                         static_cast<char*>(out), vstride, cin, cout, W, ri, ro);
    OVL_HIP(hipGetLastError());
  }
  void wgrad(const void* in, const void* gout, int cin, int cout, double2* out, int accumulate = 0) const {
    const Geo& g = u->geom.geo;
    const int nout = cin * cout * 16;
    WsBuf part(static_cast<size_t>(NPATH) * WG_BLOCKS * nout * sizeof(double2), s);
    dim3 grid(WG_BLOCKS, NPATH);
    if (recon == 18)
      hipLaunchKernelGGL(ptc_wgrad_kernel<18>, grid, dim3(256), 0, s, g, links, static_cast<const char*>(in),
                         static_cast<const char*>(gout), vstride, cin, cout, static_cast<double2*>(part.p));
    else
      hipLaunchKernelGGL(ptc_wgrad_kernel<12>, grid, dim3(256), 0, s, g, links, static_cast<const char*>(in),
                         static_cast<const char*>(gout), vstride, cin, cout, static_cast<double2*>(part.p));
    OVL_HIP(hipGetLastError());
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((nout + 255) / 256, NPATH), dim3(256), 0, s, nout, WG_BLOCKS,
                       static_cast<const double2*>(part.p), out, accumulate);
    OVL_HIP(hipGetLastError());
  }
};

size_t g_nsites(const ovl_gauge* u) { return static_cast<size_t>(u->geom.N); }

Layer make_layer(const ovl_gauge* u, hipStream_t s) {
  Layer L{u, nullptr, 0, s, spinor_vec_bytes(&u->geom, OVL_F32)};
  L.links = gauge_links(u, OVL_F32, &L.recon);
  return L;
}

}  // namespace

// out_r = M in_r for a batch of nrhs FP32 fields (back to back); the hidden
// channels of the batch come from the pool.
void net_apply(const ovl_net* net, const ovl_gauge* u, const void* in, void* out, int nrhs, hipStream_t s) {
  Layer L = make_layer(u, s);
  const int C = net->hidden;
  WsBuf hid(L.vstride * C * nrhs, s);
  WsBuf w1(net->w1.size() * sizeof(float2), s), w2(net->w2.size() * sizeof(float2), s);
  upload(net->w1, static_cast<float2*>(w1.p), s);
  upload(net->w2, static_cast<float2*>(w2.p), s);
  L.forward(in, hid.p, 1, C, static_cast<const float2*>(w1.p), nrhs);
  L.forward(hid.p, out, C, 1, static_cast<const float2*>(w2.p), nrhs);
}

}  // namespace ovl

using namespace ovl;

extern "C" {

int ovl_net_create(const ovl_geom* g, int hidden, ovl_net** out) {
  return guard([&] {
    OVL_REQUIRE(g && out, OVL_E_ARG, "null argument");
    OVL_REQUIRE(hidden >= 1 && hidden <= CMAX, OVL_E_ARG, "hidden channels must be 1..4");
    ovl_net* n = new ovl_net;
    n->geom = *g;
    n->hidden = hidden;
    n->w1.assign(static_cast<size_t>(NPATH) * hidden * 16, zc(0.0, 0.0));
    n->w2.assign(static_cast<size_t>(NPATH) * hidden * 16, zc(0.0, 0.0));
    *out = n;
    return OVL_OK;
  });
}

int ovl_net_destroy(ovl_net* n) {
  delete n;
  return OVL_OK;
}

int ovl_net_set_weights(ovl_net* n, const double* w1, const double* w2) {
  return guard([&] {
    OVL_REQUIRE(n && w1 && w2, OVL_E_ARG, "null argument");
    for (size_t i = 0; i < n->w1.size(); ++i) n->w1[i] = zc(w1[2 * i], w1[2 * i + 1]);
    for (size_t i = 0; i < n->w2.size(); ++i) n->w2[i] = zc(w2[2 * i], w2[2 * i + 1]);
    return OVL_OK;
  });
}

int ovl_net_get_weights(const ovl_net* n, double* w1, double* w2) {
  return guard([&] {
    OVL_REQUIRE(n && w1 && w2, OVL_E_ARG, "null argument");
    for (size_t i = 0; i < n->w1.size(); ++i) {
      w1[2 * i] = n->w1[i].real();
      w1[2 * i + 1] = n->w1[i].imag();
    }
    for (size_t i = 0; i < n->w2.size(); ++i) {
      w2[2 * i] = n->w2[i].real();
      w2[2 * i + 1] = n->w2[i].imag();
    }
    return OVL_OK;
  });
}

int ovl_ptc_layer_forward(const ovl_gauge* u, const void* in, int cin, void* out, int cout, const double* W,
                          ovl_stream_t st) {
  return guard([&] {
    OVL_REQUIRE(u && in && out && W, OVL_E_ARG, "null argument");
    OVL_REQUIRE(cin >= 1 && cin <= CMAX && cout >= 1 && cout <= CMAX, OVL_E_ARG, "channels must be 1..4");
    OVL_REQUIRE(in != out, OVL_E_ALIAS, "output must not alias the input");
    hipStream_t s = static_cast<hipStream_t>(st);
    Layer L = make_layer(u, s);
    const size_t nw = static_cast<size_t>(NPATH) * cin * cout * 16;
    std::vector<zc> w(nw);
    for (size_t i = 0; i < nw; ++i) w[i] = zc(W[2 * i], W[2 * i + 1]);
    WsBuf dw(nw * sizeof(float2), s);
    upload(w, static_cast<float2*>(dw.p), s);
    L.forward(in, out, cin, cout, static_cast<const float2*>(dw.p));
    return OVL_OK;
  });
}

int ovl_ptc_layer_backward(const ovl_gauge* u, const void* in, int cin, const void* gout, int cout, const double* W,
                           void* gin, double* gW, ovl_stream_t st) {
  return guard([&] {
    OVL_REQUIRE(u && in && gout && W, OVL_E_ARG, "null argument");
    OVL_REQUIRE(cin >= 1 && cin <= CMAX && cout >= 1 && cout <= CMAX && cin * cout <= CMAX, OVL_E_ARG,
                "channels must be 1..4 with cin*cout <= 4");
    hipStream_t s = static_cast<hipStream_t>(st);
    Layer L = make_layer(u, s);
    const size_t nw = static_cast<size_t>(NPATH) * cin * cout * 16;
    std::vector<zc> w(nw);
    for (size_t i = 0; i < nw; ++i) w[i] = zc(W[2 * i], W[2 * i + 1]);
    if (gin) {
      OVL_REQUIRE(gin != gout && gin != in, OVL_E_ALIAS, "gradient output aliases an input");
      WsBuf dw(nw * sizeof(float2), s);
      upload(adjoint_weights(w, cin, cout), static_cast<float2*>(dw.p), s);
      L.forward(gout, gin, cout, cin, static_cast<const float2*>(dw.p));
    }
    if (gW) {
      WsBuf dg(nw * sizeof(double2), s);
      L.wgrad(in, gout, cin, cout, static_cast<double2*>(dg.p));
      OVL_HIP(hipMemcpyAsync(gW, dg.p, nw * sizeof(double2), hipMemcpyDeviceToHost, s));
    }
    OVL_HIP(hipStreamSynchronize(s));
    return OVL_OK;
  });
}

int ovl_net_train(ovl_net* n, const ovl_gauge* u, const void* B, const void* X, int npairs, int epochs, int batch,
                  double lr, const int32_t* order, double* loss_history, ovl_stream_t st) {
  return guard([&] {
    OVL_REQUIRE(n && u && B && X && order, OVL_E_ARG, "null argument");
    OVL_REQUIRE(npairs >= 1 && epochs >= 1 && batch >= 1 && lr > 0.0, OVL_E_ARG, "bad training parameter");
    hipStream_t s = static_cast<hipStream_t>(st);
    Layer L = make_layer(u, s);
    const int C = n->hidden;
    const size_t vs = L.vstride;
    const size_t nw = n->w1.size();  // = n->w2.size()
    WsBuf hid(vs * C, s), out(vs, s), gout(vs, s), gh(vs * C, s);
    WsBuf dw1(nw * sizeof(float2), s), dw2(nw * sizeof(float2), s), dw2a(nw * sizeof(float2), s);
    WsBuf g1(nw * sizeof(double2), s), g2(nw * sizeof(double2), s);
    WsBuf sc(8 * sizeof(double), s);
    double* dsc = static_cast<double*>(sc.p);  // [0..1] norm tmp, [2] x2, [3] d2, [4] loss, [6..7] gscale
    const double one_m1[4] = {1.0, 0.0, -1.0, 0.0};
    WsBuf cst(4 * sizeof(double), s);
    OVL_HIP(hipMemcpyAsync(cst.p, one_m1, sizeof(one_m1), hipMemcpyHostToDevice, s));
    const double* d_one = static_cast<const double*>(cst.p);
    const double* d_m1 = d_one + 2;
    // Adam state over the real and imaginary parts of every weight
    std::vector<double> m1(4 * nw, 0.0), v1(4 * nw, 0.0);
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    int tstep = 0;
    std::vector<double2> hg(nw);
    const size_t n16 = vs / 16;
    auto norm2_into = [&](const void* x, double* dst) {
      blas_norm2(OVL_F32, n16, x, 1, vs, dsc, s);
      OVL_HIP(hipMemcpyAsync(dst, dsc, sizeof(double), hipMemcpyDeviceToDevice, s));
    };
    for (int ep = 0; ep < epochs; ++ep) {
      double zero = 0.0;
      OVL_HIP(hipMemcpyAsync(dsc + 4, &zero, sizeof(double), hipMemcpyHostToDevice, s));
      for (int b0 = 0; b0 < npairs; b0 += batch) {
        const int nb = std::min(batch, npairs - b0);
        upload(n->w1, static_cast<float2*>(dw1.p), s);
        upload(n->w2, static_cast<float2*>(dw2.p), s);
        upload(adjoint_weights(n->w2, C, 1), static_cast<float2*>(dw2a.p), s);
        blas_zero(g1.p, nw * sizeof(double2), s);
        blas_zero(g2.p, nw * sizeof(double2), s);
        for (int q = 0; q < nb; ++q) {
          const int idx = order[static_cast<size_t>(ep) * npairs + b0 + q];
          OVL_REQUIRE(idx >= 0 && idx < npairs, OVL_E_ARG, "training order index out of range");
          const char* bb = static_cast<const char*>(B) + static_cast<size_t>(idx) * vs;
          const char* xx = static_cast<const char*>(X) + static_cast<size_t>(idx) * vs;
          L.forward(bb, hid.p, 1, C, static_cast<const float2*>(dw1.p));
          L.forward(hid.p, out.p, C, 1, static_cast<const float2*>(dw2.p));
          // diff = out - x (into gout), loss and gradient scale
          blas_axpby(OVL_F32, xx, d_m1, OVL_F32, out.p, d_one, g_nsites(u), 1, s);
          norm2_into(xx, dsc + 2);
          norm2_into(out.p, dsc + 3);
          hipLaunchKernelGGL(pair_loss_kernel, dim3(1), dim3(64), 0, s, dsc + 3, dsc + 2, dsc + 4, dsc + 6);
          blas_axpby(OVL_F32, out.p, dsc + 6, OVL_F32, gout.p, nullptr, g_nsites(u), 1, s);
          // layer 2: weight gradient and input gradient; layer 1: weight gradient
          L.wgrad(hid.p, gout.p, C, 1, static_cast<double2*>(g2.p), 1);
          L.forward(gout.p, gh.p, 1, C, static_cast<const float2*>(dw2a.p));
          L.wgrad(bb, gh.p, 1, C, static_cast<double2*>(g1.p), 1);
        }
        // Adam step on the mean gradient of the batch
        ++tstep;
        for (int layer = 0; layer < 2; ++layer) {
          OVL_HIP(hipMemcpyAsync(hg.data(), layer == 0 ? g1.p : g2.p, nw * sizeof(double2), hipMemcpyDeviceToHost, s));
          OVL_HIP(hipStreamSynchronize(s));
          std::vector<zc>& W = layer == 0 ? n->w1 : n->w2;
          for (size_t i = 0; i < nw; ++i) {
            const double gr[2] = {hg[i].x / nb, hg[i].y / nb};
            double wv[2] = {W[i].real(), W[i].imag()};
            for (int c = 0; c < 2; ++c) {
              const size_t k = (layer * nw + i) * 2 + c;
              m1[k] = b1 * m1[k] + (1 - b1) * gr[c];
              v1[k] = b2 * v1[k] + (1 - b2) * gr[c] * gr[c];
              const double mh = m1[k] / (1 - std::pow(b1, tstep)), vh = v1[k] / (1 - std::pow(b2, tstep));
              wv[c] -= lr * mh / (std::sqrt(vh) + eps);
            }
            W[i] = zc(wv[0], wv[1]);
          }
        }
      }
      double loss = 0.0;
      OVL_HIP(hipMemcpyAsync(&loss, dsc + 4, sizeof(double), hipMemcpyDeviceToHost, s));
      OVL_HIP(hipStreamSynchronize(s));
      OVL_REQUIRE(std::isfinite(loss), OVL_E_NAN, "training loss is NaN or Inf");
      if (loss_history) loss_history[ep] = loss / npairs;
    }
    return OVL_OK;
  });
}

int ovl_net_apply(const ovl_net* n, const ovl_gauge* u, const void* in, void* out, ovl_stream_t st) {
  return guard([&] {
    OVL_REQUIRE(n && u && in && out, OVL_E_ARG, "null argument");
    OVL_REQUIRE(in != out, OVL_E_ALIAS, "output must not alias the input");
    net_apply(n, u, in, out, 1, static_cast<hipStream_t>(st));
    return OVL_OK;
  });
}

}  // extern "C"
