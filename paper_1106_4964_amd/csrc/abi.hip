// extern "C" entry points of libovl: argument checks, error codes, and the
// dispatch to the internal drivers.  Each function's contract is documented
// in include/ovl.h.
#include <atomic>
#include <cstdio>

#include "ops.h"

namespace ovl {

Geo make_geo(const int* d);
void neighbor_table(const ovl_geom* g, int32_t* dev, hipStream_t s);
void pack_spinor(const ovl_geom* g, const double* aos, void* out, int prec, int nrhs, hipStream_t s);
void unpack_spinor(const ovl_geom* g, const void* in, double* aos, int prec, int nrhs, hipStream_t s);
double su3_deviation(const ovl_gauge* u, hipStream_t s);
void gauge_create_master(ovl_gauge* u, const double* aos, hipStream_t s);
void gauge_set_repr(ovl_gauge* u, int prec, int recon, hipStream_t s);
void gauge_free(ovl_gauge* u);

namespace {
thread_local std::string g_last_error;

struct Pool {
  std::mutex mu;
  // (stream, bytes) -> free buffers
  std::multimap<std::pair<hipStream_t, size_t>, void*> free_list;
  std::map<void*, size_t> sizes;
};
Pool& pool() {
  static Pool* p = new Pool();  // never destroyed: buffers live until exit
  return *p;
}
}  // namespace

void set_last_error(const std::string& msg) { g_last_error = msg; }

namespace {
std::atomic<int64_t> g_stencil_launches{0}, g_stencil_vectors{0};
std::atomic<int64_t> g_mem_live{0}, g_mem_peak{0};
}
bool log_on() {
  static const bool on = [] {
    const char* e = std::getenv("OVL_LOG");
    return e && *e && *e != '0';
  }();
  return on;
}

void mem_track(int64_t delta) {
  const int64_t now = g_mem_live.fetch_add(delta) + delta;
  int64_t pk = g_mem_peak.load();
  while (now > pk && !g_mem_peak.compare_exchange_weak(pk, now)) {
  }
}
void count_stencil(int nrhs) {
  g_stencil_launches.fetch_add(1, std::memory_order_relaxed);
  g_stencil_vectors.fetch_add(nrhs, std::memory_order_relaxed);
}

void* ws_get(size_t bytes, hipStream_t s) {
  Pool& P = pool();
  {
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.free_list.find({s, bytes});
    if (it != P.free_list.end()) {
      void* p = it->second;
      P.free_list.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess || p == nullptr) {
    (void)hipGetLastError();
    throw Error(OVL_E_NOMEM, "device workspace allocation of " + std::to_string(bytes) + " bytes failed");
  }
  mem_track(static_cast<int64_t>(bytes));
  std::lock_guard<std::mutex> lk(P.mu);
  P.sizes[p] = bytes;
  return p;
}

void ws_put(void* p, hipStream_t s) {
  if (!p) return;
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  P.free_list.insert({{s, P.sizes[p]}, p});
}

void ws_retire_stream(hipStream_t from, hipStream_t to) {
  if (from == to) return;
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  std::vector<std::pair<size_t, void*>> moved;
  for (auto it = P.free_list.begin(); it != P.free_list.end();) {
    if (it->first.first == from) {
      moved.emplace_back(it->first.second, it->second);
      it = P.free_list.erase(it);
    } else {
      ++it;
    }
  }
  for (const auto& m : moved) P.free_list.insert({{to, m.first}, m.second});
}

}  // namespace ovl

using namespace ovl;

static hipStream_t S(ovl_stream_t s) { return static_cast<hipStream_t>(s); }

extern "C" {

const char* ovl_last_error(void) { return g_last_error.c_str(); }

int ovl_version(void) { return 100; }

int ovl_stencil_tune(int mode) {
  return guard([&] {
    OVL_REQUIRE(mode == 0 || mode == 1, OVL_E_ARG, "tune mode must be 0 or 1");
    set_tune_mode(mode);
    return OVL_OK;
  });
}

int ovl_stencil_shape(const ovl_geom* g, ovl_prec prec, int compress12, int nextra, int nrhs, int* shape) {
  return guard([&] {
    OVL_REQUIRE(g && shape, OVL_E_ARG, "null argument");
    for (int i = 0; i < 5; ++i) shape[i] = 0;
    stencil_shape(prec, compress12 ? 12 : 18, nextra, nrhs, 2, g->geo.Nh, shape);
    return OVL_OK;
  });
}

int ovl_stencil_set_shape(const ovl_geom* g, ovl_prec prec, int compress12, int nextra, int nrhs, const int* shape) {
  return guard([&] {
    OVL_REQUIRE(g && shape, OVL_E_ARG, "null argument");
    check_prec(prec);
    check_nrhs(nrhs);
    const int kr = shape[0], bs = shape[1], pipe = shape[2], rin = shape[3], tm = shape[4];
    OVL_REQUIRE(nextra >= 0 && nextra <= 3, OVL_E_ARG, "nextra must be 0..3");
    OVL_REQUIRE(bs == 32 || bs == 64 || bs == 128 || bs == 256, OVL_E_ARG, "bs must be 32, 64, 128 or 256");
    OVL_REQUIRE(rin == 0 || rin == 1, OVL_E_ARG, "rin must be 0 or 1");
    OVL_REQUIRE(tm >= 0 && tm <= g->dims[2], OVL_E_ARG, "tm must be 0, 1 or a slab thickness <= Lz");
    if (pipe) {
      OVL_REQUIRE(kr == 1 && rin == 0 && pipe >= 2 && pipe <= 4, OVL_E_ARG,
                  "pipelined shapes need kr = 1, rin = 0, depth 2..4");
    } else {
      OVL_REQUIRE(kr >= 1 && kr <= (prec == OVL_F64 ? 2 : 4) && nrhs % kr == 0, OVL_E_ARG,
                  "kr must divide nrhs (kr <= 4, <= 2 for FP64)");
      OVL_REQUIRE(!rin || bs * (nrhs / kr) <= 512, OVL_E_ARG, "rin shapes need bs * nrhs / kr <= 512");
    }
    for (int npar = 1; npar <= 2; ++npar)
      force_shape(prec, compress12 ? 12 : 18, nextra, nrhs, npar, g->geo.Nh, shape);
    return OVL_OK;
  });
}

int ovl_stencil_timer(int mode) {
  return guard([&] {
    OVL_REQUIRE(mode >= 0 && mode <= 2, OVL_E_ARG, "mode must be 0, 1 or 2");
    stencil_timer(mode);
    return OVL_OK;
  });
}

int ovl_stencil_timer_read(ovl_prec prec, int compress12, int nextra, int nrhs, int64_t* launches, double* total_ms) {
  return guard([&] {
    OVL_REQUIRE(launches && total_ms, OVL_E_ARG, "null argument");
    check_prec(prec);
    stencil_timer_read(prec, compress12 ? 12 : 18, nextra, nrhs, launches, total_ms);
    return OVL_OK;
  });
}

int ovl_counters(int64_t* stencil_launches, int64_t* stencil_vectors, int reset) {
  if (stencil_launches) *stencil_launches = g_stencil_launches.load();
  if (stencil_vectors) *stencil_vectors = g_stencil_vectors.load();
  if (reset) {
    g_stencil_launches = 0;
    g_stencil_vectors = 0;
  }
  return OVL_OK;
}

int ovl_mem_stats(int64_t* live_bytes, int64_t* peak_bytes, int reset_peak) {
  if (live_bytes) *live_bytes = g_mem_live.load();
  if (peak_bytes) *peak_bytes = g_mem_peak.load();
  if (reset_peak) g_mem_peak = g_mem_live.load();
  return OVL_OK;
}

// ------------------------------------------------------------------ geometry
int ovl_geom_create(const int32_t dims[4], ovl_geom** out) {
  return guard([&] {
    OVL_REQUIRE(dims && out, OVL_E_ARG, "null argument");
    int64_t n = 1;
    for (int k = 0; k < 4; ++k) {
      OVL_REQUIRE(dims[k] >= 2 && dims[k] % 2 == 0, OVL_E_DIMS, "lattice extents must be even and >= 2");
      n *= dims[k];
    }
    OVL_REQUIRE(n < (int64_t(1) << 31) / 8, OVL_E_DIMS, "lattice too large for 32-bit site tables");
    ovl_geom* g = new ovl_geom;
    for (int k = 0; k < 4; ++k) g->dims[k] = dims[k];
    g->N = n;
    g->geo = make_geo(g->dims);
    *out = g;
    return OVL_OK;
  });
}

int ovl_geom_destroy(ovl_geom* g) {
  delete g;
  return OVL_OK;
}

int ovl_geom_volume(const ovl_geom* g, int64_t* n) {
  return guard([&] {
    OVL_REQUIRE(g && n, OVL_E_ARG, "null argument");
    *n = g->N;
    return OVL_OK;
  });
}

int ovl_geom_eo_index(const ovl_geom* g, const int32_t c[4], int32_t* eo) {
  return guard([&] {
    OVL_REQUIRE(g && c && eo, OVL_E_ARG, "null argument");
    for (int k = 0; k < 4; ++k) OVL_REQUIRE(c[k] >= 0 && c[k] < g->dims[k], OVL_E_ARG, "coordinate out of range");
    const int64_t lex = c[0] + int64_t(g->dims[0]) * (c[1] + int64_t(g->dims[1]) * (c[2] + int64_t(g->dims[2]) * c[3]));
    const int p = (c[0] + c[1] + c[2] + c[3]) & 1;
    *eo = static_cast<int32_t>(p * (g->N / 2) + lex / 2);
    return OVL_OK;
  });
}

int ovl_geom_neighbors_device(const ovl_geom* g, int32_t* dev, ovl_stream_t s) {
  return guard([&] {
    OVL_REQUIRE(g && dev, OVL_E_ARG, "null argument");
    neighbor_table(g, dev, S(s));
    return OVL_OK;
  });
}

// ------------------------------------------------------------------- spinors
int ovl_spinor_bytes(const ovl_geom* g, ovl_prec prec, int nrhs, size_t* bytes) {
  return guard([&] {
    OVL_REQUIRE(g && bytes, OVL_E_ARG, "null argument");
    check_prec(prec);
    check_nrhs(nrhs);
    *bytes = spinor_vec_bytes(g, prec) * nrhs;
    return OVL_OK;
  });
}

int ovl_pack_spinor(const ovl_geom* g, const double* aos, void* out, ovl_prec prec, int nrhs, ovl_stream_t s) {
  return guard([&] {
    OVL_REQUIRE(g && aos && out, OVL_E_ARG, "null argument");
    check_prec(prec);
    check_nrhs(nrhs);
    OVL_REQUIRE(static_cast<const void*>(aos) != out, OVL_E_ALIAS, "pack: source and destination alias");
    pack_spinor(g, aos, out, prec, nrhs, S(s));
    return OVL_OK;
  });
}

int ovl_unpack_spinor(const ovl_geom* g, const void* in, double* aos, ovl_prec prec, int nrhs, ovl_stream_t s) {
  return guard([&] {
    OVL_REQUIRE(g && aos && in, OVL_E_ARG, "null argument");
    check_prec(prec);
    check_nrhs(nrhs);
    OVL_REQUIRE(static_cast<const void*>(aos) != in, OVL_E_ALIAS, "unpack: source and destination alias");
    unpack_spinor(g, in, aos, prec, nrhs, S(s));
    return OVL_OK;
  });
}

// --------------------------------------------------------------------- gauge
int ovl_gauge_create(const ovl_geom* g, const double* aos, ovl_stream_t s, ovl_gauge** out) {
  return guard([&] {
    OVL_REQUIRE(g && aos && out, OVL_E_ARG, "null argument");
    ovl_gauge* u = new ovl_gauge;
    u->geom = *g;
    try {
      gauge_create_master(u, aos, S(s));
    } catch (...) {
      gauge_free(u);
      delete u;
      throw;
    }
    *out = u;
    return OVL_OK;
  });
}

int ovl_gauge_set_repr(ovl_gauge* u, ovl_prec prec, int compress12, ovl_stream_t s) {
  return guard([&] {
    OVL_REQUIRE(u, OVL_E_ARG, "null argument");
    check_prec(prec);
    OVL_REQUIRE(compress12 == 0 || compress12 == 1, OVL_E_ARG, "compress12 must be 0 or 1");
    if (compress12) {
      const double dev = su3_deviation(u, S(s));
      if (!(dev <= 1e-12)) {
        char buf[128];
        snprintf(buf, sizeof buf, "12-real compression needs SU(3) links; max deviation %.3e", dev);
        throw Error(OVL_E_NOT_SU3, buf);
      }
    }
    gauge_set_repr(u, prec, compress12 ? 12 : 18, S(s));
    return OVL_OK;
  });
}

int ovl_gauge_destroy(ovl_gauge* u) {
  if (u) {
    gauge_free(u);
    delete u;
  }
  return OVL_OK;
}

const ovl_geom* ovl_gauge_geom(const ovl_gauge* u) { return u ? &u->geom : nullptr; }

// ----------------------------------------------------------------- operators
static void stencil_common(StencilArgs& A, const ovl_gauge* u, void* out, const void* in, int prec, int nrhs,
                           int* recon) {
  OVL_REQUIRE(u && out && in, OVL_E_ARG, "null argument");
  check_prec(prec);
  check_nrhs(nrhs);
  OVL_REQUIRE(out != in, OVL_E_ALIAS, "output must not alias the input");
  A = StencilArgs{};
  A.g = u->geom.geo;
  A.out = out;
  A.in = in;
  A.links = gauge_links(u, prec, recon);
  A.vstride = spinor_vec_bytes(&u->geom, prec);
}

int ovl_dslash(void* out, const void* in, const ovl_gauge* u, double m, int parity, ovl_prec prec, int nrhs,
               ovl_stream_t s) {
  return guard([&] {
    StencilArgs A;
    int recon = 0;
    stencil_common(A, u, out, in, prec, nrhs, &recon);
    OVL_REQUIRE(parity >= 0 && parity <= 2, OVL_E_ARG, "parity must be 0, 1 or 2");
    A.a = 4.0 + m;
    A.b = -0.5;
    A.par0 = parity == 2 ? 0 : parity;
    A.npar = parity == 2 ? 2 : 1;
    launch_stencil(A, prec, recon, nrhs, S(s));
    return OVL_OK;
  });
}

int ovl_hw_apply(void* out, const void* in, const ovl_gauge* u, double rho, ovl_prec prec, int nrhs,
                 ovl_stream_t s) {
  return guard([&] {
    StencilArgs A;
    int recon = 0;
    stencil_common(A, u, out, in, prec, nrhs, &recon);
    A.a = 4.0 - rho;
    A.b = -0.5;
    A.g5 = 1;
    A.par0 = 0;
    A.npar = 2;
    launch_stencil(A, prec, recon, nrhs, S(s));
    return OVL_OK;
  });
}

// --------------------------------------------------------------------- BLAS1
static size_t n16_of(const ovl_geom* g, int prec) { return spinor_vec_bytes(g, prec) / 16; }

static void blas_common(const ovl_geom* g, int prec, int nrhs) {
  OVL_REQUIRE(g, OVL_E_ARG, "null geometry");
  check_prec(prec);
  check_nrhs(nrhs);
}

int ovl_axpy(const ovl_geom* g, const double* a, const void* x, void* y, ovl_prec prec, int nrhs, ovl_stream_t s) {
  return guard([&] {
    blas_common(g, prec, nrhs);
    OVL_REQUIRE(a && x && y, OVL_E_ARG, "null argument");
    WsBuf dev(2 * sizeof(double) * nrhs, S(s));
    OVL_HIP(hipMemcpyAsync(dev.p, a, 2 * sizeof(double) * nrhs, hipMemcpyHostToDevice, S(s)));
    blas_axpy(prec, n16_of(g, prec), static_cast<double*>(dev.p), x, y, nrhs, spinor_vec_bytes(g, prec), S(s));
    OVL_HIP(hipStreamSynchronize(S(s)));  // host scalars: keep `a` alive for the copy
    return OVL_OK;
  });
}

int ovl_xpay(const ovl_geom* g, const void* x, const double* a, void* y, ovl_prec prec, int nrhs, ovl_stream_t s) {
  return guard([&] {
    blas_common(g, prec, nrhs);
    OVL_REQUIRE(a && x && y, OVL_E_ARG, "null argument");
    WsBuf dev(2 * sizeof(double) * nrhs, S(s));
    OVL_HIP(hipMemcpyAsync(dev.p, a, 2 * sizeof(double) * nrhs, hipMemcpyHostToDevice, S(s)));
    blas_xpay(prec, n16_of(g, prec), x, static_cast<double*>(dev.p), y, nrhs, spinor_vec_bytes(g, prec), S(s));
    OVL_HIP(hipStreamSynchronize(S(s)));
    return OVL_OK;
  });
}

int ovl_dot(const ovl_geom* g, const void* x, const void* y, ovl_prec prec, int nrhs, double* result,
            ovl_stream_t s) {
  return guard([&] {
    blas_common(g, prec, nrhs);
    OVL_REQUIRE(x && y && result, OVL_E_ARG, "null argument");
    WsBuf dev(2 * sizeof(double) * nrhs, S(s));
    blas_dot(prec, n16_of(g, prec), x, y, nrhs, spinor_vec_bytes(g, prec), static_cast<double*>(dev.p), S(s));
    OVL_HIP(hipMemcpyAsync(result, dev.p, 2 * sizeof(double) * nrhs, hipMemcpyDeviceToHost, S(s)));
    OVL_HIP(hipStreamSynchronize(S(s)));
    return OVL_OK;
  });
}

int ovl_norm2(const ovl_geom* g, const void* x, ovl_prec prec, int nrhs, double* result, ovl_stream_t s) {
  return guard([&] {
    blas_common(g, prec, nrhs);
    OVL_REQUIRE(x && result, OVL_E_ARG, "null argument");
    WsBuf dev(2 * sizeof(double) * nrhs, S(s));
    blas_norm2(prec, n16_of(g, prec), x, nrhs, spinor_vec_bytes(g, prec), static_cast<double*>(dev.p), S(s));
    std::vector<double> tmp(2 * nrhs);
    OVL_HIP(hipMemcpyAsync(tmp.data(), dev.p, 2 * sizeof(double) * nrhs, hipMemcpyDeviceToHost, S(s)));
    OVL_HIP(hipStreamSynchronize(S(s)));
    for (int r = 0; r < nrhs; ++r) result[r] = tmp[2 * r];
    return OVL_OK;
  });
}

int ovl_convert(const ovl_geom* g, const void* src, ovl_prec sp, void* dst, ovl_prec dp, int nrhs, ovl_stream_t s) {
  return guard([&] {
    OVL_REQUIRE(g && src && dst, OVL_E_ARG, "null argument");
    check_prec(sp);
    check_prec(dp);
    check_nrhs(nrhs);
    OVL_REQUIRE(src != dst, OVL_E_ALIAS, "convert: source and destination alias");
    blas_convert(sp, src, dp, dst, static_cast<size_t>(g->N), nrhs, S(s));
    return OVL_OK;
  });
}

}  // extern "C"
