// libovfem: C ABI of the OVFEM voxel stepper (see include/ovfem.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <limits>
#include <stdexcept>
#include <string>
#include <vector>

#include "ovfem.h"
#include "kernels.hpp"

using namespace ovfem;

namespace {

thread_local std::string g_last_error;

struct Error : std::runtime_error {
  ovfem_status code;
  Error(ovfem_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define OVFEM_HIP(expr)                                                                       \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      throw Error(e_ == hipErrorOutOfMemory ? OVFEM_ENOMEM : OVFEM_EDEVICE,                   \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                        \
    }                                                                                         \
  } while (0)

inline void require(bool ok, const std::string& msg, ovfem_status code = OVFEM_EINVAL) {
  if (!ok) throw Error(code, msg);
}

template <class F>
ovfem_status guarded(F&& f) {
  try {
    f();
    g_last_error.clear();
    return OVFEM_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return OVFEM_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return OVFEM_EDEVICE;
  }
}

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  void alloc(size_t count) {
    free();
    if (count == 0) count = 1;
    OVFEM_HIP(hipMalloc(&p, count * sizeof(T)));
    n = count;
  }
  void free() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

// Largest eigenvalue of a symmetric n x n matrix (cyclic Jacobi, host, small n).
double max_eigenvalue(std::vector<double> a, int n) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += a[p * n + q] * a[p * n + q];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        const double tt = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(tt * tt + 1.0), s = tt * c;
        for (int k = 0; k < n; ++k) {
          const double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
      }
  }
  double m = -std::numeric_limits<double>::infinity();
  for (int i = 0; i < n; ++i) m = std::max(m, a[i * n + i]);
  return m;
}

// INT8 A fragments (bf16): lane l of row tile t holds A[i = l % 16][k = 8 (l / 16) .. + 7]
// of the 16 x 32 tile.  Row i of tile t is output s = 4 t + i % 4 for in-plane corner
// G = i / 4: s < 6 are rows of AL, s >= 6 rows of AM, at corner G + 4 ((s % 6) / 3)
// and component s % 3.  Column k is (node k / 4, component k % 4), component 3 padding.
// Entries are integers of magnitude <= 98, exact in bf16.
std::vector<uint32_t> make_alane() {
  std::vector<uint32_t> out(3 * 64 * 4);
  for (int t = 0; t < 3; ++t)
    for (int l = 0; l < 64; ++l) {
      const int i = l % 16, kg = l / 16;
      const int G = i / 4, s = 4 * t + i % 4;
      const int which = s / 6, dk = (s % 6) / 3, c = s % 3;
      const int m = 3 * (G + 4 * dk) + c;
      for (int q = 0; q < 8; ++q) {
        const int k = 8 * kg + q, node = k / 4, cp = k % 4;
        int v = 0;
        if (cp < 3) v = which == 0 ? kRef.AL[m][3 * node + cp] : kRef.AM[m][3 * node + cp];
        const float f = (float)v;
        uint32_t bits;
        std::memcpy(&bits, &f, 4);
        const uint32_t bf = bits >> 16;  // exact: |v| <= 127 has <= 7 significant bits
        out[(t * 64 + l) * 4 + q / 2] |= bf << (16 * (q % 2));
      }
    }
  return out;
}

// I8 A fragments: the same matrix entries as make_alane(), as int8 bytes.
std::vector<uint64_t> make_alane8() {
  std::vector<uint64_t> out(3 * 64, 0);
  for (int t = 0; t < 3; ++t)
    for (int l = 0; l < 64; ++l) {
      const int i = l % 16, kg = l / 16;
      const int G = i / 4, s = 4 * t + i % 4;
      const int which = s / 6, dk = (s % 6) / 3, c = s % 3;
      const int m = 3 * (G + 4 * dk) + c;
      for (int q = 0; q < 8; ++q) {
        const int k = 8 * kg + q, node = k / 4, cp = k % 4;
        int v = 0;
        if (cp < 3) v = which == 0 ? kRef.AL[m][3 * node + cp] : kRef.AM[m][3 * node + cp];
        out[t * 64 + l] |= (uint64_t)(uint8_t)(int8_t)v << (8 * q);
      }
    }
  return out;
}

bool valid_precision(int p) { return p == OVFEM_FP64 || p == OVFEM_INT8 || p == OVFEM_INT8_I32; }

}  // namespace

struct ovfem_solver {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t nx = 0, ny = 0, nz = 0;
  double h = 0;
  int n_shots = 1;
  int precision = OVFEM_FP64;
  Geom geom{};
  size_t n_nodes = 0, n_elem = 0;

  DevBuf<double> u[2];
  int cur = 0;  // u[cur] = u^n, u[cur ^ 1] = u^{n-1}
  DevBuf<double> mat, acoef;  // mat: [element][2] = (h lam / 256, h mu / 128)
  DevBuf<int> expo[2], expo_tmp;
  int exp_cur = 0;
  bool exp_valid = false;
  DevBuf<uint32_t> alane;
  DevBuf<uint64_t> alane8;

  DevBuf<int> src_ptr, src_node, src_comp, src_row;
  DevBuf<double> wavelet;
  int src_nt = 0, n_src = 0;
  DevBuf<int> rec_ptr, rec_node, rec_idx;
  DevBuf<double> traces;
  int rec_nt = 0, n_rec = 0;

  // adjoint: forward checkpoints (u^s, u^{s-1}) at s = 0, every, 2 every, ... since reset
  int64_t ckpt_every = 0, ckpt_slots = 0;
  DevBuf<double> ckpt;           // [slot][2][3 n_nodes]
  bool ckpt_valid = false;       // the run since reset was checkpointed with this precision
  int ckpt_precision = OVFEM_FP64;

  std::vector<double> mass;      // nodal mass (host)
  std::vector<uint8_t> fixed;    // nodal fixed flags (host)
  bool model_set = false, dt_set = false, acoef_dirty = true;
  double dt = 0, dt_bound = 0;
  int64_t step = 0;

  ~ovfem_solver() {
    (void)hipStreamSynchronize(stream);
    u[0].free();
    u[1].free();
    mat.free();
    acoef.free();
    expo[0].free();
    expo[1].free();
    expo_tmp.free();
    alane.free();
    alane8.free();
    src_ptr.free();
    src_node.free();
    src_comp.free();
    src_row.free();
    wavelet.free();
    rec_ptr.free();
    rec_node.free();
    rec_idx.free();
    traces.free();
    ckpt.free();
  }

  double* ckpt_u(int64_t slot, int which) { return ckpt.p + (size_t)(2 * slot + which) * 3 * n_nodes; }

  int tile_of(int64_t X, int64_t Y, int64_t Z) const {
    return (int)(X / TN + geom.tiles_x * (Y / TN + geom.tiles_y * (Z / geom.tz)));
  }

  void check_device() {
    int d = -1;
    OVFEM_HIP(hipGetDevice(&d));
    require(d == device, "solver used on a different current device than it was created on", OVFEM_ESTATE);
  }

  void refresh_acoef() {
    if (!acoef_dirty) return;
    std::vector<double> a(n_nodes, 0.0);
    for (size_t i = 0; i < n_nodes; ++i)
      if (!fixed[i] && mass[i] > 0.0) a[i] = dt * dt / mass[i];
    OVFEM_HIP(hipMemcpyAsync(acoef.p, a.data(), n_nodes * sizeof(double), hipMemcpyHostToDevice, stream));
    OVFEM_HIP(hipStreamSynchronize(stream));
    acoef_dirty = false;
  }

  void launch_exponents(const double* v, int* dst) {
    ovfem_exponent_kernel<<<geom.n_wg, NTHR, 0, stream>>>(geom, v, dst);
    OVFEM_HIP(hipGetLastError());
  }

  KArgs base_args() const {
    KArgs A{};
    A.g = geom;
    A.mat = mat.p;
    A.acoef = acoef.p;
    A.alane = reinterpret_cast<const v4u*>(alane.p);
    A.alane8 = alane8.p;
    A.src_ptr = src_ptr.p;
    A.src_node = src_node.p;
    A.src_comp = src_comp.p;
    A.src_row = src_row.p;
    A.wavelet = wavelet.p;
    A.src_nt = src_nt;
    A.rec_ptr = rec_ptr.p;
    A.rec_node = rec_node.p;
    A.rec_idx = rec_idx.p;
    A.traces = traces.p;
    A.rec_nt = rec_nt;
    return A;
  }

  void launch_layer(const KArgs& A, int mode) {
    const dim3 grid(geom.n_wg), block(NTHR);
    if (precision == OVFEM_FP64) {
      if (mode == MODE_STEP)
        ovfem_layer_kernel<PATH_FP64, MODE_STEP><<<grid, block, 0, stream>>>(A);
      else
        ovfem_layer_kernel<PATH_FP64, MODE_MATVEC><<<grid, block, 0, stream>>>(A);
    } else if (precision == OVFEM_INT8) {
      if (mode == MODE_STEP)
        ovfem_layer_kernel<PATH_INT8, MODE_STEP><<<grid, block, 0, stream>>>(A);
      else
        ovfem_layer_kernel<PATH_INT8, MODE_MATVEC><<<grid, block, 0, stream>>>(A);
    } else {
      if (mode == MODE_STEP)
        ovfem_layer_kernel<PATH_I8, MODE_STEP><<<grid, block, 0, stream>>>(A);
      else
        ovfem_layer_kernel<PATH_I8, MODE_MATVEC><<<grid, block, 0, stream>>>(A);
    }
    OVFEM_HIP(hipGetLastError());
  }

  void zero_state() {
    OVFEM_HIP(hipMemsetAsync(u[0].p, 0, 3 * n_nodes * sizeof(double), stream));
    OVFEM_HIP(hipMemsetAsync(u[1].p, 0, 3 * n_nodes * sizeof(double), stream));
    if (traces.p) OVFEM_HIP(hipMemsetAsync(traces.p, 0, traces.n * sizeof(double), stream));
    cur = 0;
    step = 0;
    launch_exponents(u[cur].p, expo[exp_cur].p);
    exp_valid = true;
    ckpt_valid = ckpt_every > 0;
    ckpt_precision = precision;
  }

  void do_steps(int64_t n) {
    require(model_set, "ovfem_step: model not set", OVFEM_ESTATE);
    require(dt_set, "ovfem_step: dt not set", OVFEM_ESTATE);
    refresh_acoef();
    if (!exp_valid) {
      launch_exponents(u[cur].p, expo[exp_cur].p);
      exp_valid = true;
    }
    KArgs A = base_args();
    if (ckpt_valid && precision != ckpt_precision) ckpt_valid = false;
    for (int64_t i = 0; i < n; ++i) {
      if (ckpt_valid && step % ckpt_every == 0) {
        const int64_t slot = step / ckpt_every;
        if (slot < ckpt_slots) {
          const size_t bytes = 3 * n_nodes * sizeof(double);
          OVFEM_HIP(hipMemcpyAsync(ckpt_u(slot, 0), u[cur].p, bytes, hipMemcpyDeviceToDevice, stream));
          OVFEM_HIP(hipMemcpyAsync(ckpt_u(slot, 1), u[cur ^ 1].p, bytes, hipMemcpyDeviceToDevice, stream));
        } else {
          ckpt_valid = false;  // ran past the checkpoint capacity
        }
      }
      A.u = u[cur].p;
      A.uprev = u[cur ^ 1].p;
      A.unext = u[cur ^ 1].p;
      A.exp_in = expo[exp_cur].p;
      A.exp_out = expo[exp_cur ^ 1].p;
      A.step = step;
      launch_layer(A, MODE_STEP);
      cur ^= 1;
      exp_cur ^= 1;
      ++step;
    }
  }
};

extern "C" {

int32_t ovfem_version(void) { return 100; }

const char* ovfem_last_error(void) { return g_last_error.c_str(); }

ovfem_status ovfem_create(ovfem_solver** out, int64_t nx, int64_t ny, int64_t nz, double h, int32_t n_shots,
                          int32_t precision, void* stream) {
  return guarded([&] {
    require(out != nullptr, "ovfem_create: out is NULL");
    *out = nullptr;
    require(nx > 0 && ny > 0 && nz > 0, "ovfem_create: grid sizes must be positive");
    require(std::isfinite(h) && h > 0, "ovfem_create: h must be positive");
    require(n_shots == 1, "ovfem_create: n_shots must be 1");
    require(valid_precision(precision), "ovfem_create: unknown precision");
    const double nn = double(nx + 1) * double(ny + 1) * double(nz + 1);
    require(nn < 2147483647.0, "ovfem_create: more than 2^31 - 1 nodes");
    auto s = new ovfem_solver();
    try {
      OVFEM_HIP(hipGetDevice(&s->device));
      s->stream = reinterpret_cast<hipStream_t>(stream);
      s->nx = nx;
      s->ny = ny;
      s->nz = nz;
      s->h = h;
      s->precision = precision;
      s->n_nodes = (size_t)(nx + 1) * (ny + 1) * (nz + 1);
      s->n_elem = (size_t)nx * ny * nz;
      Geom& g = s->geom;
      g.nx = (int)nx;
      g.ny = (int)ny;
      g.nz = (int)nz;
      g.tiles_x = (int)((nx + 1 + TN - 1) / TN);
      g.tiles_y = (int)((ny + 1 + TN - 1) / TN);
      g.chunks = (int)((nz + 1 + 15) / 16);
      g.tz = (int)((nz + 1 + g.chunks - 1) / g.chunks);
      g.chunks = (int)((nz + 1 + g.tz - 1) / g.tz);
      g.n_wg = g.tiles_x * g.tiles_y * g.chunks;
      s->u[0].alloc(3 * s->n_nodes);
      s->u[1].alloc(3 * s->n_nodes);
      s->mat.alloc(2 * s->n_elem);
      s->acoef.alloc(s->n_nodes);
      s->expo[0].alloc(g.n_wg);
      s->expo[1].alloc(g.n_wg);
      s->expo_tmp.alloc(g.n_wg);
      auto al = make_alane();
      s->alane.alloc(al.size());
      OVFEM_HIP(hipMemcpyAsync(s->alane.p, al.data(), al.size() * 4, hipMemcpyHostToDevice, s->stream));
      auto al8 = make_alane8();
      s->alane8.alloc(al8.size());
      OVFEM_HIP(hipMemcpyAsync(s->alane8.p, al8.data(), al8.size() * 8, hipMemcpyHostToDevice, s->stream));
      std::vector<int> zeros(g.n_wg + 1, 0);
      s->src_ptr.alloc(g.n_wg + 1);
      s->rec_ptr.alloc(g.n_wg + 1);
      OVFEM_HIP(hipMemcpyAsync(s->src_ptr.p, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice, s->stream));
      OVFEM_HIP(hipMemcpyAsync(s->rec_ptr.p, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice, s->stream));
      s->src_node.alloc(1);
      s->src_comp.alloc(1);
      s->src_row.alloc(1);
      s->wavelet.alloc(1);
      s->rec_node.alloc(1);
      s->rec_idx.alloc(1);
      s->traces.alloc(1);
      s->mass.assign(s->n_nodes, 0.0);
      s->fixed.assign(s->n_nodes, 0);
      s->zero_state();
      OVFEM_HIP(hipStreamSynchronize(s->stream));
    } catch (...) {
      delete s;
      throw;
    }
    *out = s;
  });
}

ovfem_status ovfem_destroy(ovfem_solver* s) {
  return guarded([&] { delete s; });
}

ovfem_status ovfem_set_precision(ovfem_solver* s, int32_t precision) {
  return guarded([&] {
    require(s != nullptr, "ovfem_set_precision: solver is NULL");
    require(valid_precision(precision), "ovfem_set_precision: unknown precision");
    s->precision = precision;
  });
}

ovfem_status ovfem_set_model(ovfem_solver* s, const double* lam, const double* mu, const double* rho,
                             const uint8_t* solid) {
  return guarded([&] {
    require(s != nullptr, "ovfem_set_model: solver is NULL");
    require(lam && mu && rho, "ovfem_set_model: lam, mu and rho must be non-NULL host arrays");
    s->check_device();
    const size_t ne = s->n_elem;
    const int64_t nx = s->nx, ny = s->ny, nz = s->nz;
    const double h = s->h;
    std::vector<double> mt(2 * ne), mass(s->n_nodes, 0.0);
    // stability: largest eigenvalues of the two reference matrices
    std::vector<double> al(576), am(576);
    for (int i = 0; i < 24; ++i)
      for (int j = 0; j < 24; ++j) {
        al[i * 24 + j] = kRef.AL[i][j] / 256.0;
        am[i * 24 + j] = kRef.AM[i][j] / 128.0;
      }
    const double el = max_eigenvalue(al, 24), em = max_eigenvalue(am, 24);
    double wmax2 = 0.0;
    for (int64_t k = 0; k < nz; ++k)
      for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i) {
          const size_t e = (size_t)(i + nx * (j + ny * k));
          const bool sol = solid == nullptr || solid[e] != 0;
          if (!sol) {
            mt[2 * e] = mt[2 * e + 1] = 0.0;
            continue;
          }
          const double L = lam[e], M = mu[e], R = rho[e];
          require(std::isfinite(L) && std::isfinite(M) && std::isfinite(R),
                  "ovfem_set_model: non-finite material in element " + std::to_string(e));
          require(M > 0 && L + 2.0 * M / 3.0 > 0 && R > 0,
                  "ovfem_set_model: need mu > 0, lam + 2 mu / 3 > 0, rho > 0 (element " + std::to_string(e) + ")");
          mt[2 * e] = h * L / 256.0;
          mt[2 * e + 1] = h * M / 128.0;
          const double me = R * h * h * h / 8.0;
          // lambda_max(lam K_lam + mu K_mu) <= max(lam, 0) lambda_max(K_lam) + mu lambda_max(K_mu)
          wmax2 = std::max(wmax2, h * (std::max(L, 0.0) * el + M * em) / me);
          for (int dk = 0; dk < 2; ++dk)
            for (int dj = 0; dj < 2; ++dj)
              for (int di = 0; di < 2; ++di)
                mass[(size_t)((i + di) + (nx + 1) * ((j + dj) + (ny + 1) * (k + dk)))] += me;
        }
    s->dt_bound = wmax2 > 0 ? 2.0 / std::sqrt(wmax2) : std::numeric_limits<double>::infinity();
    OVFEM_HIP(hipMemcpyAsync(s->mat.p, mt.data(), 2 * ne * sizeof(double), hipMemcpyHostToDevice, s->stream));
    OVFEM_HIP(hipStreamSynchronize(s->stream));
    s->mass.swap(mass);
    s->model_set = true;
    s->acoef_dirty = true;
    if (s->dt_set && s->dt > s->dt_bound) s->dt_set = false;  // dt must be set again
    s->zero_state();
  });
}

ovfem_status ovfem_set_fixed_nodes(ovfem_solver* s, const uint8_t* fixed) {
  return guarded([&] {
    require(s != nullptr, "ovfem_set_fixed_nodes: solver is NULL");
    if (fixed)
      std::memcpy(s->fixed.data(), fixed, s->n_nodes);
    else
      std::fill(s->fixed.begin(), s->fixed.end(), 0);
    s->acoef_dirty = true;
  });
}

ovfem_status ovfem_set_dt(ovfem_solver* s, double dt) {
  return guarded([&] {
    require(s != nullptr, "ovfem_set_dt: solver is NULL");
    require(s->model_set, "ovfem_set_dt: set the model first", OVFEM_ESTATE);
    require(std::isfinite(dt) && dt > 0, "ovfem_set_dt: dt must be positive");
    require(dt <= s->dt_bound, "ovfem_set_dt: dt = " + std::to_string(dt) +
                                   " exceeds the element stability bound " + std::to_string(s->dt_bound));
    s->dt = dt;
    s->dt_set = true;
    s->acoef_dirty = true;
  });
}

ovfem_status ovfem_set_sources(ovfem_solver* s, int32_t n, const int64_t* node, const int32_t* comp,
                               const int32_t* shot, const double* wavelet, int64_t nt) {
  return guarded([&] {
    require(s != nullptr, "ovfem_set_sources: solver is NULL");
    require(n >= 0, "ovfem_set_sources: n < 0");
    require(n == 0 || (node && comp && wavelet && nt > 0), "ovfem_set_sources: missing arrays or nt <= 0");
    require((double)n * (double)std::max<int64_t>(nt, 1) < 2147483647.0, "ovfem_set_sources: table too large");
    const int nwg = s->geom.n_wg;
    std::vector<std::vector<int>> per(nwg);
    for (int i = 0; i < n; ++i) {
      require(node[i] >= 0 && (size_t)node[i] < s->n_nodes, "ovfem_set_sources: node out of range");
      require(comp[i] >= 0 && comp[i] < 3, "ovfem_set_sources: comp out of range");
      require(shot == nullptr || (shot[i] >= 0 && shot[i] < s->n_shots), "ovfem_set_sources: shot out of range");
      const int64_t X = node[i] % (s->nx + 1), Y = (node[i] / (s->nx + 1)) % (s->ny + 1),
                    Z = node[i] / ((s->nx + 1) * (s->ny + 1));
      per[s->tile_of(X, Y, Z)].push_back(i);
    }
    std::vector<int> ptr(nwg + 1, 0), nd, cp, row;
    for (int w = 0; w < nwg; ++w) {
      ptr[w + 1] = ptr[w] + (int)per[w].size();
      for (int i : per[w]) {
        nd.push_back((int)node[i]);
        cp.push_back(comp[i]);
        row.push_back(i);
      }
    }
    DevBuf<int> dptr, dnd, dcp, drow;
    DevBuf<double> dw;
    dptr.alloc(nwg + 1);
    dnd.alloc(nd.size());
    dcp.alloc(cp.size());
    drow.alloc(row.size());
    dw.alloc((size_t)n * (size_t)std::max<int64_t>(nt, 1));
    OVFEM_HIP(hipMemcpyAsync(dptr.p, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice, s->stream));
    if (n > 0) {
      OVFEM_HIP(hipMemcpyAsync(dnd.p, nd.data(), nd.size() * 4, hipMemcpyHostToDevice, s->stream));
      OVFEM_HIP(hipMemcpyAsync(dcp.p, cp.data(), cp.size() * 4, hipMemcpyHostToDevice, s->stream));
      OVFEM_HIP(hipMemcpyAsync(drow.p, row.data(), row.size() * 4, hipMemcpyHostToDevice, s->stream));
      OVFEM_HIP(hipMemcpyAsync(dw.p, wavelet, (size_t)n * nt * sizeof(double), hipMemcpyHostToDevice, s->stream));
    }
    OVFEM_HIP(hipStreamSynchronize(s->stream));
    std::swap(s->src_ptr, dptr);
    std::swap(s->src_node, dnd);
    std::swap(s->src_comp, dcp);
    std::swap(s->src_row, drow);
    std::swap(s->wavelet, dw);
    dptr.free();
    dnd.free();
    dcp.free();
    drow.free();
    dw.free();
    s->n_src = n;
    s->src_nt = n > 0 ? (int)nt : 0;
  });
}

ovfem_status ovfem_set_receivers(ovfem_solver* s, int32_t n, const int64_t* node, int64_t nt_max) {
  return guarded([&] {
    require(s != nullptr, "ovfem_set_receivers: solver is NULL");
    require(n >= 0 && nt_max >= 0, "ovfem_set_receivers: negative count");
    require(n == 0 || node, "ovfem_set_receivers: node is NULL");
    require((double)n * 3.0 * (double)nt_max < 2147483647.0 * 4.0, "ovfem_set_receivers: trace buffer too large");
    const int nwg = s->geom.n_wg;
    std::vector<std::vector<int>> per(nwg);
    for (int i = 0; i < n; ++i) {
      require(node[i] >= 0 && (size_t)node[i] < s->n_nodes, "ovfem_set_receivers: node out of range");
      const int64_t X = node[i] % (s->nx + 1), Y = (node[i] / (s->nx + 1)) % (s->ny + 1),
                    Z = node[i] / ((s->nx + 1) * (s->ny + 1));
      per[s->tile_of(X, Y, Z)].push_back(i);
    }
    std::vector<int> ptr(nwg + 1, 0), nd, idx;
    for (int w = 0; w < nwg; ++w) {
      ptr[w + 1] = ptr[w] + (int)per[w].size();
      for (int i : per[w]) {
        nd.push_back((int)node[i]);
        idx.push_back(i);
      }
    }
    DevBuf<int> dptr, dnd, didx;
    DevBuf<double> dtr;
    dptr.alloc(nwg + 1);
    dnd.alloc(nd.size());
    didx.alloc(idx.size());
    dtr.alloc((size_t)s->n_shots * n * 3 * nt_max);
    OVFEM_HIP(hipMemcpyAsync(dptr.p, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice, s->stream));
    if (n > 0) {
      OVFEM_HIP(hipMemcpyAsync(dnd.p, nd.data(), nd.size() * 4, hipMemcpyHostToDevice, s->stream));
      OVFEM_HIP(hipMemcpyAsync(didx.p, idx.data(), idx.size() * 4, hipMemcpyHostToDevice, s->stream));
    }
    OVFEM_HIP(hipMemsetAsync(dtr.p, 0, dtr.n * sizeof(double), s->stream));
    OVFEM_HIP(hipStreamSynchronize(s->stream));
    std::swap(s->rec_ptr, dptr);
    std::swap(s->rec_node, dnd);
    std::swap(s->rec_idx, didx);
    std::swap(s->traces, dtr);
    dptr.free();
    dnd.free();
    didx.free();
    dtr.free();
    s->n_rec = n;
    s->rec_nt = (int)nt_max;
  });
}

ovfem_status ovfem_reset(ovfem_solver* s) {
  return guarded([&] {
    require(s != nullptr, "ovfem_reset: solver is NULL");
    s->check_device();
    s->zero_state();
  });
}

ovfem_status ovfem_step(ovfem_solver* s, int64_t n) {
  return guarded([&] {
    require(s != nullptr, "ovfem_step: solver is NULL");
    require(n >= 0, "ovfem_step: n < 0");
    s->check_device();
    s->do_steps(n);
  });
}

ovfem_status ovfem_matvec(ovfem_solver* s, const double* u, double* Ku) {
  return guarded([&] {
    require(s != nullptr, "ovfem_matvec: solver is NULL");
    require(u && Ku, "ovfem_matvec: NULL array");
    require(s->model_set, "ovfem_matvec: model not set", OVFEM_ESTATE);
    const size_t bytes = 3 * s->n_nodes * sizeof(double);
    const char *a = (const char*)u, *b = (const char*)Ku;
    require(a + bytes <= b || b + bytes <= a, "ovfem_matvec: u and Ku overlap");
    s->check_device();
    KArgs A = s->base_args();
    A.u = u;
    A.ku = Ku;
    if (s->precision != OVFEM_FP64) {
      s->launch_exponents(u, s->expo_tmp.p);
      A.exp_in = s->expo_tmp.p;
    }
    s->launch_layer(A, MODE_MATVEC);
  });
}

ovfem_status ovfem_get_wavefield(ovfem_solver* s, int32_t which, double* out) {
  return guarded([&] {
    require(s != nullptr, "ovfem_get_wavefield: solver is NULL");
    require(which == 0 || which == 1, "ovfem_get_wavefield: which must be 0 or 1");
    require(out != nullptr, "ovfem_get_wavefield: out is NULL");
    const int src = which == 0 ? s->cur : s->cur ^ 1;
    OVFEM_HIP(hipMemcpyAsync(out, s->u[src].p, 3 * s->n_nodes * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    OVFEM_HIP(hipStreamSynchronize(s->stream));
  });
}

ovfem_status ovfem_set_wavefield(ovfem_solver* s, const double* un, const double* unm1, int64_t step) {
  return guarded([&] {
    require(s != nullptr, "ovfem_set_wavefield: solver is NULL");
    require(un && unm1, "ovfem_set_wavefield: NULL array");
    require(step >= 0, "ovfem_set_wavefield: step < 0");
    s->check_device();
    const size_t bytes = 3 * s->n_nodes * sizeof(double);
    OVFEM_HIP(hipMemcpyAsync(s->u[s->cur].p, un, bytes, hipMemcpyDeviceToDevice, s->stream));
    OVFEM_HIP(hipMemcpyAsync(s->u[s->cur ^ 1].p, unm1, bytes, hipMemcpyDeviceToDevice, s->stream));
    s->launch_exponents(s->u[s->cur].p, s->expo[s->exp_cur].p);
    s->exp_valid = true;
    s->step = step;
    s->ckpt_valid = false;
    OVFEM_HIP(hipStreamSynchronize(s->stream));
  });
}

ovfem_status ovfem_get_traces(ovfem_solver* s, double* out) {
  return guarded([&] {
    require(s != nullptr, "ovfem_get_traces: solver is NULL");
    require(out != nullptr || s->n_rec == 0 || s->rec_nt == 0, "ovfem_get_traces: out is NULL");
    const size_t n = (size_t)s->n_shots * s->n_rec * 3 * s->rec_nt;
    if (n > 0)
      OVFEM_HIP(hipMemcpyAsync(out, s->traces.p, n * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    OVFEM_HIP(hipStreamSynchronize(s->stream));
  });
}

ovfem_status ovfem_get_step(ovfem_solver* s, int64_t* step) {
  return guarded([&] {
    require(s != nullptr && step != nullptr, "ovfem_get_step: NULL argument");
    *step = s->step;
  });
}

ovfem_status ovfem_set_checkpointing(ovfem_solver* s, int64_t every, int64_t max_steps) {
  return guarded([&] {
    require(s != nullptr, "ovfem_set_checkpointing: solver is NULL");
    require(every >= 0 && max_steps >= 0, "ovfem_set_checkpointing: negative argument");
    s->check_device();
    DevBuf<double> buf;
    int64_t slots = 0;
    if (every > 0) {
      slots = max_steps / every + 1;
      buf.alloc((size_t)slots * 2 * 3 * s->n_nodes);
    }
    OVFEM_HIP(hipStreamSynchronize(s->stream));
    std::swap(s->ckpt, buf);
    buf.free();
    s->ckpt_every = every;
    s->ckpt_slots = slots;
    s->zero_state();
    OVFEM_HIP(hipStreamSynchronize(s->stream));
  });
}

ovfem_status ovfem_adjoint(ovfem_solver* s, const double* residual, double* g_lam, double* g_mu) {
  return guarded([&] {
    require(s != nullptr, "ovfem_adjoint: solver is NULL");
    require(residual && g_lam && g_mu, "ovfem_adjoint: NULL array");
    s->check_device();
    const int64_t n = s->step;
    require(s->ckpt_valid && s->ckpt_every > 0,
            "ovfem_adjoint: the forward run since reset was not checkpointed (call ovfem_set_checkpointing, "
            "then step from reset without changing precision or wavefield)", OVFEM_ESTATE);
    require(n >= 1, "ovfem_adjoint: no forward steps to differentiate", OVFEM_ESTATE);
    require(s->n_rec > 0 && n <= s->rec_nt, "ovfem_adjoint: receivers must record every forward step", OVFEM_ESTATE);
    require(s->model_set && s->dt_set, "ovfem_adjoint: model and dt not set", OVFEM_ESTATE);
    s->refresh_acoef();
    const int64_t every = s->ckpt_every;
    const size_t vec = 3 * s->n_nodes;
    const Geom& g = s->geom;

    // adjoint sources: every receiver component, with the residual as its force
    std::vector<int> rec_node_h(s->n_rec), rec_idx_h(s->n_rec), rec_ptr_h(g.n_wg + 1);
    OVFEM_HIP(hipMemcpy(rec_node_h.data(), s->rec_node.p, s->n_rec * 4, hipMemcpyDeviceToHost));
    OVFEM_HIP(hipMemcpy(rec_idx_h.data(), s->rec_idx.p, s->n_rec * 4, hipMemcpyDeviceToHost));
    OVFEM_HIP(hipMemcpy(rec_ptr_h.data(), s->rec_ptr.p, (g.n_wg + 1) * 4, hipMemcpyDeviceToHost));
    std::vector<int> aptr(g.n_wg + 1, 0), anode, acomp, arow;
    for (int w = 0; w < g.n_wg; ++w) {
      for (int r = rec_ptr_h[w]; r < rec_ptr_h[w + 1]; ++r)
        for (int c = 0; c < 3; ++c) {
          anode.push_back(rec_node_h[r]);
          acomp.push_back(c);
          arow.push_back(3 * rec_idx_h[r] + c);
        }
      aptr[w + 1] = (int)anode.size();
    }
    DevBuf<int> d_aptr, d_anode, d_acomp, d_arow;
    DevBuf<double> seg, wbuf, zeros;
    DevBuf<int> fexp, wexp;
    d_aptr.alloc(aptr.size());
    d_anode.alloc(anode.size());
    d_acomp.alloc(acomp.size());
    d_arow.alloc(arow.size());
    seg.alloc((size_t)(every + 1) * vec);
    wbuf.alloc(2 * vec);
    fexp.alloc(2 * g.n_wg);
    wexp.alloc(2 * g.n_wg);
    auto free_all = [&] {
      d_aptr.free(); d_anode.free(); d_acomp.free(); d_arow.free();
      seg.free(); wbuf.free(); fexp.free(); wexp.free();
    };
    try {
      OVFEM_HIP(hipMemcpyAsync(d_aptr.p, aptr.data(), aptr.size() * 4, hipMemcpyHostToDevice, s->stream));
      OVFEM_HIP(hipMemcpyAsync(d_anode.p, anode.data(), anode.size() * 4, hipMemcpyHostToDevice, s->stream));
      OVFEM_HIP(hipMemcpyAsync(d_acomp.p, acomp.data(), acomp.size() * 4, hipMemcpyHostToDevice, s->stream));
      OVFEM_HIP(hipMemcpyAsync(d_arow.p, arow.data(), arow.size() * 4, hipMemcpyHostToDevice, s->stream));
      OVFEM_HIP(hipMemsetAsync(g_lam, 0, s->n_elem * sizeof(double), s->stream));
      OVFEM_HIP(hipMemsetAsync(g_mu, 0, s->n_elem * sizeof(double), s->stream));
      OVFEM_HIP(hipMemsetAsync(wbuf.p, 0, 2 * vec * sizeof(double), s->stream));
      double* w[2] = {wbuf.p, wbuf.p + vec};
      int wc = 0, we = 0;  // w[wc] = w^{m+1}, w[wc ^ 1] = w^{m+2}
      s->launch_exponents(w[0], wexp.p);

      KArgs F = s->base_args();  // forward recompute: forward sources, no receivers
      F.rec_nt = 0;
      KArgs B = s->base_args();  // adjoint steps: residual injected at the receivers
      B.src_ptr = d_aptr.p;
      B.src_node = d_anode.p;
      B.src_comp = d_acomp.p;
      B.src_row = d_arow.p;
      B.wavelet = residual;
      B.src_nt = s->rec_nt;
      B.rec_nt = 0;
      const int gblocks = (int)((s->n_elem + NTHR - 1) / NTHR);

      for (int64_t sg = (n - 1) / every; sg >= 0; --sg) {
        const int64_t s0 = sg * every, e0 = std::min(s0 + every, n);
        // state(k) = u^{s0+k}: slot 0 and u^{s0-1} from the checkpoint, the rest recomputed
        auto state = [&](int64_t k) -> double* {
          if (k < 0) return s->ckpt_u(sg, 1);
          if (k == 0) return s->ckpt_u(sg, 0);
          return seg.p + (size_t)k * vec;
        };
        int fe = 0;
        s->launch_exponents(state(0), fexp.p);
        for (int64_t t = s0; t < e0; ++t) {
          F.u = state(t - s0);
          F.uprev = state(t - s0 - 1);
          F.unext = state(t - s0 + 1);
          F.exp_in = fexp.p + fe * g.n_wg;
          F.exp_out = fexp.p + (fe ^ 1) * g.n_wg;
          F.step = t;
          s->launch_layer(F, MODE_STEP);
          fe ^= 1;
        }
        for (int64_t m = e0; m > s0; --m) {
          B.u = w[wc];
          B.uprev = w[wc ^ 1];
          B.unext = w[wc ^ 1];
          B.exp_in = wexp.p + we * g.n_wg;
          B.exp_out = wexp.p + (we ^ 1) * g.n_wg;
          B.step = m - 1;
          s->launch_layer(B, MODE_STEP);
          wc ^= 1;
          we ^= 1;
          ovfem_gradient_kernel<<<gblocks, NTHR, 0, s->stream>>>(g, s->h, s->mat.p, state(m - 1 - s0), w[wc], g_lam,
                                                                 g_mu);
          OVFEM_HIP(hipGetLastError());
        }
      }
      OVFEM_HIP(hipStreamSynchronize(s->stream));
    } catch (...) {
      (void)hipStreamSynchronize(s->stream);
      free_all();
      throw;
    }
    free_all();
  });
}

ovfem_status ovfem_synchronize(ovfem_solver* s) {
  return guarded([&] {
    require(s != nullptr, "ovfem_synchronize: solver is NULL");
    OVFEM_HIP(hipStreamSynchronize(s->stream));
  });
}

}  // extern "C"
