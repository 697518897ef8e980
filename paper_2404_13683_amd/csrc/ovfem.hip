// libovfem: C ABI of the OVFEM voxel stepper (declarations and contracts in ovfem.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <limits>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "adjoint.hpp"
#include "launch.hpp"
#include "ovfem.h"

using namespace ovfem;

namespace {

thread_local std::string g_last_error;

struct Error : std::runtime_error {
  ovfem_status code;
  Error(ovfem_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// A failed HIP call also leaves its error as the runtime's last error, which the next
// hipGetLastError() (after a later, good launch) would report again: it is consumed here.
#define OVFEM_HIP(expr)                                                                       \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      (void)hipGetLastError();                                                                \
      throw Error(e_ == hipErrorOutOfMemory ? OVFEM_ENOMEM : OVFEM_EDEVICE,                   \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                        \
    }                                                                                         \
  } while (0)

inline void require(bool ok, const std::string& msg, ovfem_status code = OVFEM_EINVAL) {
  if (!ok) throw Error(code, msg);
}

// Per block: 1 if any of its values of v is not finite (NaN or infinite), else 0.  One
// plain store per block; the host ORs the block flags.
constexpr int kFiniteBlocks = 1024;
__global__ void nonfinite_kernel(const double* v, size_t n, int* flags) {
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  int bad = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    bad |= !isfinite(v[i]);
  if (bad) any = 1;
  __syncthreads();
  if (threadIdx.x == 0) flags[blockIdx.x] = any;
}

// Deterministic pseudo-random values in [-scale, scale) (splitmix64 of the index): the
// wavefield the autotuner times on, so that candidates run on data of a real run's
// statistics rather than on the all-zero state of a fresh solver.
__global__ void fill_random_kernel(double* v, size_t n, unsigned long long seed, double scale) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned long long z = (unsigned long long)i + seed * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  v[i] = scale * ((double)(z >> 11) * 0x1p-52 - 1.0);
}

// *p = v (a device step base set in stream order, without a host value to keep alive).
__global__ void set_step_kernel(long long* p, long long v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
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

// Device buffer; freed explicitly by its holder (swapped, never copied implicitly).
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

template <class T>
void upload(DevBuf<T>& dst, const std::vector<T>& src, hipStream_t stream) {
  dst.alloc(src.size());
  if (!src.empty())
    OVFEM_HIP(hipMemcpyAsync(dst.p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, stream));
}

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

// Matrix-core A operands: lane l of row tile t holds A[i = l % 16][k = 8 (l / 16) .. + 7]
// of the 16 x 32 tile.  Row i of tile t is output s = 4 t + i % 4 for in-plane corner
// G = i / 4: s < 6 are rows of AL, s >= 6 rows of AM, at corner G + 4 ((s % 6) / 3)
// and component s % 3.  Column k is (node k / 4, component k % 4), component 3 padding.
int alane_entry(int elem, int t, int l, int q) {
  const int i = l % 16, kg = l / 16;
  const int G = i / 4, s = 4 * t + i % 4;
  const int which = s / 6, dk = (s % 6) / 3, c = s % 3;
  const int m = 3 * (G + 4 * dk) + c;
  const int k = 8 * kg + q, node = k / 4, cp = k % 4;
  if (cp == 3) return 0;
  const int n = 3 * node + cp;
  if (elem == OVFEM_ELEMENT_TRILINEAR) return which == 0 ? kTri.AL[m][n] : kTri.AM[m][n];
  return which == 0 ? kRef.AL[m][n] : kRef.AM[m][n];
}

// bf16 form, two entries per 32-bit word: |entry| <= 127 has at most 7 significant
// bits, so the upper half of its FP32 encoding is exact.
std::vector<uint32_t> make_alane_bf16(int elem) {
  std::vector<uint32_t> out(3 * 64 * 4, 0);
  for (int t = 0; t < 3; ++t)
    for (int l = 0; l < 64; ++l)
      for (int q = 0; q < 8; ++q) {
        const float f = (float)alane_entry(elem, t, l, q);
        uint32_t bits;
        std::memcpy(&bits, &f, 4);
        out[(t * 64 + l) * 4 + q / 2] |= (bits >> 16) << (16 * (q % 2));
      }
  return out;
}

// int8 form, eight entries per 64-bit word.
std::vector<uint64_t> make_alane_i8(int elem) {
  std::vector<uint64_t> out(3 * 64, 0);
  for (int t = 0; t < 3; ++t)
    for (int l = 0; l < 64; ++l)
      for (int q = 0; q < 8; ++q)
        out[t * 64 + l] |= (uint64_t)(uint8_t)(int8_t)alane_entry(elem, t, l, q) << (8 * q);
  return out;
}

bool valid_precision(int p) {
  return p == OVFEM_FP64 || p == OVFEM_INT8 || p == OVFEM_INT8_BF16 || p == OVFEM_FP64_SF;
}

// Element-product form: precision and, for OVFEM_INT8, the digit stage count.
struct Form {
  int precision;
  int stages;
  bool damp;  // Rayleigh-damped step kernels
  int elem;   // OVFEM_ELEMENT_*: selects the FP64 path's compile-time element matrices
  int ty;     // tile height in element rows (16 or 32)
};

// One record, one work-group per tile (and shot).
template <int MODE>
void launch_unit(Form f, const KArgs& A, const long long* base, long long step, hipStream_t stream) {
  const bool d = MODE == MODE_STEP && f.damp;
  if (f.precision == OVFEM_FP64) {
    if (f.elem == OVFEM_ELEMENT_TRILINEAR)
      launch_tiles<PATH_FP64, 8, 1>(f.ty, MODE, d, A, base, step, stream);
    else
      launch_tiles<PATH_FP64, 8, 0>(f.ty, MODE, d, A, base, step, stream);
  } else if (f.precision == OVFEM_INT8) {
    switch (f.stages) {
      case 4: launch_tiles<PATH_INT8, 4, 0>(f.ty, MODE, d, A, base, step, stream); break;
      case 5: launch_tiles<PATH_INT8, 5, 0>(f.ty, MODE, d, A, base, step, stream); break;
      case 6: launch_tiles<PATH_INT8, 6, 0>(f.ty, MODE, d, A, base, step, stream); break;
      case 7: launch_tiles<PATH_INT8, 7, 0>(f.ty, MODE, d, A, base, step, stream); break;
      default: launch_tiles<PATH_INT8, 8, 0>(f.ty, MODE, d, A, base, step, stream); break;
    }
  } else if (f.precision == OVFEM_FP64_SF) {
    if (f.elem == OVFEM_ELEMENT_TRILINEAR)
      launch_tiles<PATH_FP64SF, 8, 1>(f.ty, MODE, d, A, base, step, stream);
    else
      launch_tiles<PATH_FP64SF, 8, 0>(f.ty, MODE, d, A, base, step, stream);
  } else {
    launch_tiles<PATH_BF16, 8, 0>(f.ty, MODE, d, A, base, step, stream);
  }
  OVFEM_HIP(hipGetLastError());
}

// Many units in one launch; grid_cap > 0 caps the grid (rounded down to a multiple of
// 8, at least 8) so that the work-groups stride over the work list.
void launch_units(Form f, const KArgs* units, const int* begin, int n_units, int total, int grid_cap,
                  const long long* base, long long step, hipStream_t stream) {
  int grid = total;
  if (grid_cap > 0 && grid_cap < total) grid = std::max(8, (grid_cap / 8) * 8);
  const bool d = f.damp;
  if (f.precision == OVFEM_FP64) {
    if (f.elem == OVFEM_ELEMENT_TRILINEAR)
      launch_list<PATH_FP64, 8, 1>(f.ty, d, grid, units, begin, n_units, total, base, step, stream);
    else
      launch_list<PATH_FP64, 8, 0>(f.ty, d, grid, units, begin, n_units, total, base, step, stream);
  } else if (f.precision == OVFEM_INT8) {
    switch (f.stages) {
      case 4: launch_list<PATH_INT8, 4, 0>(f.ty, d, grid, units, begin, n_units, total, base, step, stream); break;
      case 5: launch_list<PATH_INT8, 5, 0>(f.ty, d, grid, units, begin, n_units, total, base, step, stream); break;
      case 6: launch_list<PATH_INT8, 6, 0>(f.ty, d, grid, units, begin, n_units, total, base, step, stream); break;
      case 7: launch_list<PATH_INT8, 7, 0>(f.ty, d, grid, units, begin, n_units, total, base, step, stream); break;
      default: launch_list<PATH_INT8, 8, 0>(f.ty, d, grid, units, begin, n_units, total, base, step, stream); break;
    }
  } else if (f.precision == OVFEM_FP64_SF) {
    if (f.elem == OVFEM_ELEMENT_TRILINEAR)
      launch_list<PATH_FP64SF, 8, 1>(f.ty, d, grid, units, begin, n_units, total, base, step, stream);
    else
      launch_list<PATH_FP64SF, 8, 0>(f.ty, d, grid, units, begin, n_units, total, base, step, stream);
  } else {
    launch_list<PATH_BF16, 8, 0>(f.ty, d, grid, units, begin, n_units, total, base, step, stream);
  }
  OVFEM_HIP(hipGetLastError());
}

// Tiling: 15 x 15 owned node columns per work-group, node planes split into chunks of
// equal depth close to chunk_planes.
Geom make_geom(int64_t nx, int64_t ny, int64_t nz, int chunk_planes, int ty) {
  Geom g{};
  g.nx = (int)nx;
  g.ny = (int)ny;
  g.nz = (int)nz;
  g.ty = ty;
  g.tiles_x = (int)((nx + 1 + TN - 1) / TN);
  g.tiles_y = (int)((ny + 1 + (ty - 1) - 1) / (ty - 1));
  const int64_t target = std::max(1, chunk_planes);
  g.chunks = (int)((nz + 1 + target - 1) / target);
  g.tz = (int)((nz + 1 + g.chunks - 1) / g.chunks);
  g.chunks = (int)((nz + 1 + g.tz - 1) / g.tz);
  g.n_wg = g.tiles_x * g.tiles_y * g.chunks;
  return g;
}

// Per-tile CSR tables of sources (per shot) and receivers (shared by the shots).
struct SourceTables {
  DevBuf<int> ptr, node, comp, row;
  void free() {
    for (auto* b : {&ptr, &node, &comp, &row}) b->free();
  }
};
struct ReceiverTables {
  DevBuf<int> ptr, node, idx;
  void free() {
    for (auto* b : {&ptr, &node, &idx}) b->free();
  }
};

}  // namespace

struct ovfem_solver {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t nx = 0, ny = 0, nz = 0;
  double h = 0;
  int n_shots = 1;
  int precision = OVFEM_FP64;
  int stages = 8;  // digit stages M of OVFEM_INT8
  int element = OVFEM_ELEMENT_OVFEM;
  Geom geom{};
  size_t n_nodes = 0, n_elem = 0;

  // state, [shot][node][3] per buffer: at phase ph, u^n is u[buf_cur(ph)] and u^{n-1} is
  // u[buf_prev(ph)]; a step writes u^{n+1} into u[buf_next(ph)] and moves to phase
  // buf_next(ph).  Undamped: two buffers, u^{n+1} over u^{n-1}.  Damped: three
  // (neighbouring work-groups still read the halo of u^{n-1}).
  DevBuf<double> u[3];
  int phase = 0;
  double alpha = 0.0, beta = 0.0;  // Rayleigh damping C = alpha M + beta K
  DevBuf<double> mat, acoef;     // mat: [element][2] = (h lam / 256, h mu / 128)
  DevBuf<uint32_t> alane_bf16;
  DevBuf<uint64_t> alane_i8;

  SourceTables src;              // ptr: [shot][n_wg + 1]
  DevBuf<double> wavelet;        // [n_src][src_nt]
  int src_nt = 0, n_src = 0;
  std::vector<int64_t> src_node_h;
  std::vector<int32_t> src_comp_h, src_shot_h;
  ReceiverTables rec;
  DevBuf<double> traces;         // [shot][rec][3][rec_nt]
  int rec_nt = 0, n_rec = 0;
  std::vector<int64_t> rec_node_h;

  std::vector<double> mass;      // nodal mass (host)
  std::vector<uint8_t> fixed;    // nodal fixed flags (host)
  bool model_set = false, dt_set = false, acoef_dirty = true;
  double dt = 0, wmax2 = 0;      // wmax2: upper bound of the squared angular frequencies
  int64_t step = 0;

  // adjoint: forward checkpoints (u^s, u^{s-1}) at s = 0, every, 2 every, ... since reset
  int64_t ckpt_every = 0, ckpt_slots = 0;
  DevBuf<double> ckpt;           // [slot][2][3 n_nodes]
  bool ckpt_valid = false;       // the run since reset was checkpointed with this form
  int ckpt_form = -1;

  // launch configuration
  int chunk_planes = 16, persist_groups = 0, graph_steps = 0;
  DevBuf<KArgs> units;           // [phase][shot]: arguments of each shot at each phase
  DevBuf<int> unit_begin;        // [shot + 1]: first work item of each shot
  DevBuf<long long> step_base;   // step index of the next replay of a captured block
  bool tables_dirty = true;
  hipGraphExec_t graph[2] = {nullptr, nullptr};  // captured block starting at phase p (undamped)
  int graph_form[2] = {-1, -1};                   // precision * 16 + stages it was captured with

  ~ovfem_solver() {
    (void)hipStreamSynchronize(stream);
    drop_graphs();
    for (auto* b : {&u[0], &u[1], &u[2], &mat, &acoef, &wavelet, &traces, &ckpt}) b->free();
    unit_begin.free();
    src.free();
    rec.free();
    alane_bf16.free();
    alane_i8.free();
    units.free();
    step_base.free();
  }

  size_t vec() const { return 3 * n_nodes; }
  bool damped() const { return alpha != 0.0 || beta != 0.0; }
  int n_phase() const { return damped() ? 3 : 2; }
  int buf_cur(int ph) const { return ph; }
  int buf_prev(int ph) const { return damped() ? (ph + 2) % 3 : ph ^ 1; }
  int buf_next(int ph) const { return damped() ? (ph + 1) % 3 : ph ^ 1; }
  Form form() const { return Form{precision, stages, damped(), element, geom.ty}; }
  // kernels of this form: element, precision, stage count, tile height
  int form_code() const {
    return geom.ty * 4096 + element * 256 + precision * 16 + (precision == OVFEM_INT8 ? stages : 0);
  }
  double damp_b() const { return beta / dt; }
  double damp_a() const { return 0.5 * alpha * dt; }
  // stability of the (damped) recursion for the largest mode: w^2 dt (dt + 2 beta) <= 4
  double dt_limit(double b) const {
    return wmax2 > 0 ? -b + std::sqrt(b * b + 4.0 / wmax2) : std::numeric_limits<double>::infinity();
  }
  // u^{slot every} (which = 0) or u^{slot every - 1} (which = 1) of the checkpoint store.
  // every > 1: pairs [slot][which]; every = 1: one tape of states u^{-1}, u^0, u^1, ...
  // that the forward run steps through directly (no copies)
  double* ckpt_u(int64_t slot, int which) {
    const size_t all = (size_t)n_shots * vec();  // every shot's nodal vector, [shot][node][3]
    if (ckpt_every == 1) return ckpt.p + (size_t)(slot + 1 - which) * all;
    return ckpt.p + (size_t)(2 * slot + which) * all;
  }

  void check_device() {
    int d = -1;
    OVFEM_HIP(hipGetDevice(&d));
    require(d == device, "solver used on a different current device than it was created on", OVFEM_ESTATE);
  }

  void drop_graphs() {
    for (int p = 0; p < 2; ++p) {
      if (graph[p]) (void)hipGraphExecDestroy(graph[p]);
      graph[p] = nullptr;
      graph_form[p] = -1;
    }
  }
  // launch arguments changed (pointers, tiling, sources, receivers)
  void invalidate_launches() {
    tables_dirty = true;
    drop_graphs();
  }

  static int tile_of(const Geom& g, int64_t node) {
    const int64_t X = node % (g.nx + 1), Y = (node / (g.nx + 1)) % (g.ny + 1),
                  Z = node / ((int64_t)(g.nx + 1) * (g.ny + 1));
    return (int)(X / TN + g.tiles_x * (Y / (g.ty - 1) + (int64_t)g.tiles_y * (Z / g.tz)));
  }

  void refresh_acoef() {
    if (!acoef_dirty) return;
    std::vector<double> a(n_nodes, 0.0);
    const double scale = 1.0 / (1.0 + damp_a());
    for (size_t i = 0; i < n_nodes; ++i)
      if (!fixed[i] && mass[i] > 0.0) a[i] = dt * dt / mass[i] * scale;
    OVFEM_HIP(hipMemcpyAsync(acoef.p, a.data(), n_nodes * sizeof(double), hipMemcpyHostToDevice, stream));
    OVFEM_HIP(hipStreamSynchronize(stream));
    acoef_dirty = false;
  }

  // source lists of every (shot, tile) for tiling g; rows index the wavelet table
  SourceTables build_sources(const Geom& g, const std::vector<int64_t>& node, const std::vector<int32_t>& comp,
                             const std::vector<int32_t>& shot) const {
    const int nwg = g.n_wg, S = n_shots;
    std::vector<std::vector<int>> per((size_t)S * nwg);
    for (size_t i = 0; i < node.size(); ++i) per[(size_t)shot[i] * nwg + tile_of(g, node[i])].push_back((int)i);
    std::vector<int> ptr((size_t)S * (nwg + 1), 0), nd, cp, row;
    for (int s = 0; s < S; ++s) {
      int* p = ptr.data() + (size_t)s * (nwg + 1);
      p[0] = (int)nd.size();
      for (int w = 0; w < nwg; ++w) {
        for (int i : per[(size_t)s * nwg + w]) {
          nd.push_back((int)node[i]);
          cp.push_back(comp[i]);
          row.push_back(i);
        }
        p[w + 1] = (int)nd.size();
      }
    }
    SourceTables t;
    try {
      upload(t.ptr, ptr, stream);
      upload(t.node, nd, stream);
      upload(t.comp, cp, stream);
      upload(t.row, row, stream);
      OVFEM_HIP(hipStreamSynchronize(stream));
    } catch (...) {
      t.free();
      throw;
    }
    return t;
  }

  ReceiverTables build_receivers(const Geom& g, const std::vector<int64_t>& node) const {
    const int nwg = g.n_wg;
    std::vector<std::vector<int>> per(nwg);
    for (size_t i = 0; i < node.size(); ++i) per[tile_of(g, node[i])].push_back((int)i);
    std::vector<int> ptr(nwg + 1, 0), nd, idx;
    for (int w = 0; w < nwg; ++w) {
      for (int i : per[w]) {
        nd.push_back((int)node[i]);
        idx.push_back(i);
      }
      ptr[w + 1] = (int)nd.size();
    }
    ReceiverTables t;
    try {
      upload(t.ptr, ptr, stream);
      upload(t.node, nd, stream);
      upload(t.idx, idx, stream);
      OVFEM_HIP(hipStreamSynchronize(stream));
    } catch (...) {
      t.free();
      throw;
    }
    return t;
  }

  // the arguments of one shot at phase ph
  KArgs shot_args(int shot, int ph) const {
    KArgs A{};
    const int c = buf_cur(ph), p = buf_prev(ph), x = buf_next(ph);
    A.g = geom;
    A.u = u[c].p + (size_t)shot * vec();
    A.uprev = u[p].p + (size_t)shot * vec();
    A.unext = u[x].p + (size_t)shot * vec();
    A.mat = mat.p;
    A.acoef = acoef.p;
    if (damped()) {
      const double ad = damp_a();
      A.damp_b = damp_b();
      A.damp_c1 = 2.0 / (1.0 + ad);
      A.damp_c2 = (1.0 - ad) / (1.0 + ad);
    }
    A.alane = reinterpret_cast<const v4u*>(alane_bf16.p);
    A.alane8 = alane_i8.p;
    A.src_ptr = src.ptr.p + (size_t)shot * (geom.n_wg + 1);
    A.src_node = src.node.p;
    A.src_comp = src.comp.p;
    A.src_row = src.row.p;
    A.wavelet = wavelet.p;
    A.src_nt = src_nt;
    A.rec_ptr = rec.ptr.p;
    A.rec_node = rec.node.p;
    A.rec_idx = rec.idx.p;
    A.traces = traces.p + (size_t)shot * n_rec * 3 * rec_nt;
    A.rec_nt = rec_nt;
    A.step = 0;
    return A;
  }

  void refresh_tables() {
    if (!tables_dirty) return;
    std::vector<KArgs> t((size_t)n_phase() * n_shots);
    for (int p = 0; p < n_phase(); ++p)
      for (int s = 0; s < n_shots; ++s) t[(size_t)p * n_shots + s] = shot_args(s, p);
    std::vector<int> begin(n_shots + 1);
    for (int s = 0; s <= n_shots; ++s) begin[s] = s * geom.n_wg;
    OVFEM_HIP(hipStreamSynchronize(stream));  // earlier launches may still read the old tables
    upload(units, t, stream);
    upload(unit_begin, begin, stream);
    OVFEM_HIP(hipStreamSynchronize(stream));
    tables_dirty = false;
  }

  // one step of every shot at phase ph; step index *base + step_arg.  The shots of the
  // grid share one argument record with per-shot strides, unless a grid cap asks for
  // the striding work-list kernel.
  void launch_step(hipStream_t st, int ph, const long long* base, long long step_arg) {
    if (n_shots == 1 || persist_groups == 0) {
      KArgs A = shot_args(0, ph);
      A.n_units = n_shots;
      A.unit_u = (long long)vec();
      A.unit_src = geom.n_wg + 1;
      A.unit_tr = (long long)n_rec * 3 * rec_nt;
      launch_unit<MODE_STEP>(form(), A, base, step_arg, st);
    } else {
      launch_units(form(), units.p + (size_t)ph * n_shots, unit_begin.p, n_shots, n_shots * geom.n_wg,
                   persist_groups, base, step_arg, st);
    }
  }

  // capture graph_steps (even) undamped steps starting at phase p, followed by the
  // advance of the device step base; the phase is p again after the block
  void capture_graph(int p) {
    hipStream_t cs = nullptr;
    hipGraph_t g = nullptr;
    OVFEM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    try {
      OVFEM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      try {
        for (int i = 0; i < graph_steps; ++i) launch_step(cs, p ^ (i & 1), step_base.p, i);
        ovfem_advance_step_kernel<<<1, 64, 0, cs>>>(step_base.p, graph_steps);
        OVFEM_HIP(hipGetLastError());
      } catch (...) {
        (void)hipStreamEndCapture(cs, &g);
        throw;
      }
      OVFEM_HIP(hipStreamEndCapture(cs, &g));
      OVFEM_HIP(hipGraphInstantiate(&graph[p], g, nullptr, nullptr, 0));
      graph_form[p] = form_code();
    } catch (...) {
      if (g) (void)hipGraphDestroy(g);
      (void)hipStreamDestroy(cs);
      throw;
    }
    (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
  }

  void zero_state() {
    const size_t bytes = (size_t)n_shots * vec() * sizeof(double);
    for (auto& b : u)
      if (b.p) OVFEM_HIP(hipMemsetAsync(b.p, 0, bytes, stream));
    if (traces.p) OVFEM_HIP(hipMemsetAsync(traces.p, 0, traces.n * sizeof(double), stream));
    phase = 0;
    step = 0;
    ckpt_valid = ckpt_every > 0;
    ckpt_form = form_code();
  }

  void prepare_steps() {
    require(model_set, "ovfem_step: model not set", OVFEM_ESTATE);
    require(dt_set, "ovfem_step: dt not set", OVFEM_ESTATE);
    refresh_acoef();
    refresh_tables();
  }

  void do_steps(int64_t n) {
    prepare_steps();
    if (ckpt_valid && form_code() != ckpt_form) ckpt_valid = false;
    int64_t done = 0;
    if (graph_steps > 0 && !ckpt_valid && !damped() && n >= graph_steps) {
      if (!graph[phase] || graph_form[phase] != form_code()) {
        if (graph[phase]) (void)hipGraphExecDestroy(graph[phase]);
        graph[phase] = nullptr;
        capture_graph(phase);
      }
      const long long s0 = step;
      OVFEM_HIP(hipMemcpyAsync(step_base.p, &s0, sizeof(long long), hipMemcpyHostToDevice, stream));
      OVFEM_HIP(hipStreamSynchronize(stream));  // s0 is a host stack value
      for (; done + graph_steps <= n; done += graph_steps) OVFEM_HIP(hipGraphLaunch(graph[phase], stream));
      step += done;  // an even count: the phase is unchanged
    }
    if (ckpt_valid && ckpt_every == 1) {
      // every state kept: step through the tape, u^{s+1} written straight to its slot
      // (every shot in one launch, as launch_step does without a grid cap)
      const int64_t m = std::min<int64_t>(n - done, ckpt_slots - 1 - step);
      if (m > 0) {
        const size_t bytes = (size_t)n_shots * vec() * sizeof(double);
        OVFEM_HIP(hipMemcpyAsync(ckpt_u(step, 0), u[buf_cur(phase)].p, bytes, hipMemcpyDeviceToDevice, stream));
        OVFEM_HIP(hipMemcpyAsync(ckpt_u(step, 1), u[buf_prev(phase)].p, bytes, hipMemcpyDeviceToDevice, stream));
        for (int64_t i = 0; i < m; ++i) {
          KArgs A = shot_args(0, phase);
          A.u = ckpt_u(step, 0);
          A.uprev = ckpt_u(step, 1);
          A.unext = ckpt_u(step + 1, 0);
          A.n_units = n_shots;
          A.unit_u = (long long)vec();
          A.unit_src = geom.n_wg + 1;
          A.unit_tr = (long long)n_rec * 3 * rec_nt;
          launch_unit<MODE_STEP>(form(), A, nullptr, step, stream);
          phase = buf_next(phase);
          ++step;
        }
        done += m;
        OVFEM_HIP(hipMemcpyAsync(u[buf_cur(phase)].p, ckpt_u(step, 0), bytes, hipMemcpyDeviceToDevice, stream));
        OVFEM_HIP(hipMemcpyAsync(u[buf_prev(phase)].p, ckpt_u(step, 1), bytes, hipMemcpyDeviceToDevice, stream));
      }
    }
    for (; done < n; ++done) {
      if (ckpt_valid && step % ckpt_every == 0) {
        const int64_t slot = step / ckpt_every;
        if (slot < ckpt_slots) {
          const size_t bytes = (size_t)n_shots * vec() * sizeof(double);
          OVFEM_HIP(hipMemcpyAsync(ckpt_u(slot, 0), u[buf_cur(phase)].p, bytes, hipMemcpyDeviceToDevice, stream));
          OVFEM_HIP(hipMemcpyAsync(ckpt_u(slot, 1), u[buf_prev(phase)].p, bytes, hipMemcpyDeviceToDevice, stream));
        } else {
          ckpt_valid = false;  // ran past the checkpoint capacity
        }
      }
      launch_step(stream, phase, nullptr, step);
      phase = buf_next(phase);
      ++step;
    }
  }

  // change the z-chunk depth: new tiling and tile lists; the state is kept
  void retile(int planes, int ty) {
    const Geom g = make_geom(nx, ny, nz, planes, ty);
    SourceTables st;
    ReceiverTables rt;
    try {
      st = build_sources(g, src_node_h, src_comp_h, src_shot_h);
      rt = build_receivers(g, rec_node_h);
    } catch (...) {
      st.free();
      rt.free();
      throw;
    }
    OVFEM_HIP(hipStreamSynchronize(stream));
    std::swap(src, st);
    std::swap(rec, rt);
    st.free();
    rt.free();
    geom = g;
    chunk_planes = planes;
    ckpt_valid = false;  // INT8 results depend on the tiling (the staging exponent's blocks)
    invalidate_launches();
    OVFEM_HIP(hipStreamSynchronize(stream));
  }
};

// Argument tables of a batched launch.  Table q holds every unit's arguments for the
// batch steps B with B % kBatchTables == q (a member's buffer phase cycles with period 2,
// or 3 when damped), and each unit's step offset: its member's step minus the batch's.
// While the members advance only through the batch the tables stay the same from one
// call to the next, so they are uploaded again only when a member was changed or stepped
// alone.
constexpr int kBatchTables = 6;

struct ovfem_batch {
  std::vector<ovfem_solver*> members;
  hipStream_t stream = nullptr;
  int persist_groups = 0;
  long long steps = 0;         // batch steps taken (B of the next step)
  std::vector<KArgs> t_host;   // the tables as last uploaded, [B mod 6][unit]
  std::vector<int> begin_host; // [unit + 1]: first work item of each unit
  DevBuf<KArgs> units;
  DevBuf<int> begin;
  std::vector<KArgs> t_fixed;  // host side of ovfem_batch_step_noalloc's tables (capacity kept)
  std::vector<int> begin_fixed;
  // captured blocks of graph_steps (a multiple of kBatchTables) batch steps starting at a
  // batch step B = 0 (mod kBatchTables), replayed with the step base in device memory
  int graph_steps = 0;
  hipGraphExec_t graph = nullptr;
  const KArgs* graph_units = nullptr;  // the tables and launch shape the graph was captured with
  int graph_n_units = -1, graph_total = -1, graph_persist = -1, graph_form = -1;
  DevBuf<long long> step_base;
  ~ovfem_batch() {
    (void)hipStreamSynchronize(stream);
    drop_graph();
    units.free();
    begin.free();
    step_base.free();
  }
  void drop_graph() {
    if (graph) (void)hipGraphExecDestroy(graph);
    graph = nullptr;
    graph_units = nullptr;
  }

  // capture graph_steps launches at B = base + i, B = i (mod kBatchTables), then the
  // advance of the base
  void capture(const KArgs* units_d, const int* begin_d, int n_units, int total) {
    drop_graph();
    if (!step_base.p) step_base.alloc(1);
    const Form form = members[0]->form();
    hipStream_t cs = nullptr;
    hipGraph_t g = nullptr;
    OVFEM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    try {
      OVFEM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      try {
        for (int i = 0; i < graph_steps; ++i)
          launch_units(form, units_d + (size_t)(i % kBatchTables) * n_units, begin_d, n_units, total, persist_groups,
                       step_base.p, i, cs);
        ovfem_advance_step_kernel<<<1, 64, 0, cs>>>(step_base.p, graph_steps);
        OVFEM_HIP(hipGetLastError());
      } catch (...) {
        (void)hipStreamEndCapture(cs, &g);
        throw;
      }
      OVFEM_HIP(hipStreamEndCapture(cs, &g));
      OVFEM_HIP(hipGraphInstantiate(&graph, g, nullptr, nullptr, 0));
    } catch (...) {
      if (g) (void)hipGraphDestroy(g);
      (void)hipStreamDestroy(cs);
      throw;
    }
    (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    graph_units = units_d;
    graph_n_units = n_units;
    graph_total = total;
    graph_persist = persist_groups;
    graph_form = members[0]->form_code();
  }

  // validate the members for a batched launch; returns the work-item count
  double check_members() const {
    double items = 0;
    for (auto* m : members) {
      require(m->form_code() == members[0]->form_code(), "ovfem_batch_step: members differ in precision, stages or tile rows",
              OVFEM_ESTATE);
      require(m->damped() == members[0]->damped(),
              "ovfem_batch_step: damped and undamped members cannot share a batch", OVFEM_ESTATE);
      m->check_device();
      items += (double)m->n_shots * m->geom.n_wg;
    }
    require(items < 2147483647.0, "ovfem_batch_step: too many work items");
    return items;
  }

  // the tables for batch steps from `steps` on (t: [B mod 6][unit], begin: [unit + 1])
  void tables(std::vector<KArgs>& t, std::vector<int>& bg) const {
    bg.assign(1, 0);
    for (auto* m : members)
      for (int s = 0; s < m->n_shots; ++s) bg.push_back(bg.back() + m->geom.n_wg);
    const size_t n_units = bg.size() - 1;
    t.assign((size_t)kBatchTables * n_units, KArgs{});
    const int q0 = (int)(steps % kBatchTables);
    size_t v = 0;
    for (auto* m : members)
      for (int s = 0; s < m->n_shots; ++s, ++v)
        for (int q = 0; q < kBatchTables; ++q) {
          int ph = m->phase;  // phase at the next batch step; then advance to a step with B % 6 == q
          for (int i = 0; i < (q - q0 + kBatchTables) % kBatchTables; ++i) ph = m->buf_next(ph);
          KArgs A = m->shot_args(s, ph);
          A.step = m->step - steps;
          std::memcpy(&t[(size_t)q * n_units + v], &A, sizeof(KArgs));  // padding stays zero
        }
  }

  // enqueue n steps reading the device tables units_d / begin_d (bg: the host copy of
  // begin_d), then advance the members.  With use_graph, whole blocks of graph_steps
  // steps that start at B = 0 (mod kBatchTables) are replayed from a captured graph.
  void launch(const KArgs* units_d, const int* begin_d, const std::vector<int>& bg, int64_t n, bool use_graph) {
    const Form form = members[0]->form();
    const int n_units = (int)bg.size() - 1, total = bg.back();
    int64_t i = 0;
    auto plain = [&](int64_t upto) {
      for (; i < upto; ++i) {
        const long long B = steps + i;
        launch_units(form, units_d + (size_t)(B % kBatchTables) * n_units, begin_d, n_units, total, persist_groups,
                     nullptr, B, stream);
      }
    };
    if (use_graph && graph_steps > 0 && !form.damp) {
      const int64_t lead = (kBatchTables - steps % kBatchTables) % kBatchTables;
      if (n - lead >= graph_steps) {
        plain(lead);
        const int code = members[0]->form_code();
        if (!graph || graph_units != units_d || graph_n_units != n_units || graph_total != total ||
            graph_persist != persist_groups || graph_form != code)
          capture(units_d, begin_d, n_units, total);
        set_step_kernel<<<1, 64, 0, stream>>>(step_base.p, steps + i);
        OVFEM_HIP(hipGetLastError());
        for (; i + graph_steps <= n; i += graph_steps) OVFEM_HIP(hipGraphLaunch(graph, stream));
      }
    }
    plain(n);
    for (auto* m : members) {
      for (int64_t i = 0; i < n % m->n_phase(); ++i) m->phase = m->buf_next(m->phase);
      m->step += n;
      m->ckpt_valid = false;
    }
    steps += n;
  }
};

// Device memory of ovfem_batch_step_noalloc: a fixed array in the code object, one copy
// per device, held until the process ends.  Host code must not pass its name to a kernel
// or a copy (it is a host-side stand-in); scratch_address() gives each device's address.
static __device__ __align__(256) unsigned char scratch[OVFEM_NOALLOC_SCRATCH_BYTES];
static_assert((OVFEM_NOALLOC_SCRATCH_BYTES - sizeof(int)) / (kBatchTables * sizeof(KArgs) + sizeof(int)) == 702,
              "ovfem.h states the unit limit of ovfem_batch_step_noalloc");

namespace {
std::mutex g_scratch_mutex;
std::vector<unsigned char*> g_scratch_address;  // [device]

// The current device's address of `scratch`, looked up once per device with that device
// current.
unsigned char* scratch_address() {
  int device = -1;
  OVFEM_HIP(hipGetDevice(&device));
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if ((int)g_scratch_address.size() <= device) g_scratch_address.resize(device + 1, nullptr);
  if (!g_scratch_address[device]) {
    void* p = nullptr;
    OVFEM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    require(p != nullptr, "ovfem_batch_step_noalloc: no device address for the scratch array", OVFEM_EDEVICE);
    g_scratch_address[device] = static_cast<unsigned char*>(p);
  }
  return g_scratch_address[device];
}
}  // namespace

extern "C" {

int32_t ovfem_version(void) { return 200; }

const char* ovfem_last_error(void) { return g_last_error.c_str(); }

ovfem_status ovfem_create(ovfem_solver** out, int64_t nx, int64_t ny, int64_t nz, double h, int32_t n_shots,
                          int32_t precision, void* stream) {
  return guarded([&] {
    require(out != nullptr, "ovfem_create: out is NULL");
    *out = nullptr;
    require(nx > 0 && ny > 0 && nz > 0, "ovfem_create: grid sizes must be positive");
    require(std::isfinite(h) && h > 0, "ovfem_create: h must be positive");
    require(n_shots >= 1 && n_shots <= OVFEM_MAX_SHOTS, "ovfem_create: n_shots out of range");
    require(valid_precision(precision), "ovfem_create: unknown precision");
    const double nn = double(nx + 1) * double(ny + 1) * double(nz + 1);
    require(nn < 2147483647.0, "ovfem_create: more than 2^31 - 1 nodes");
    // the kernels address a node plane ([node][3] doubles) and an element layer ([element][2]
    // doubles) with 32-bit byte offsets
    require(24.0 * double(nx + 1) * double(ny + 1) < 4294967296.0,
            "ovfem_create: more than 2^32 / 24 nodes in one z plane");
    auto s = new ovfem_solver();
    try {
      OVFEM_HIP(hipGetDevice(&s->device));
      s->stream = reinterpret_cast<hipStream_t>(stream);
      s->nx = nx;
      s->ny = ny;
      s->nz = nz;
      s->h = h;
      s->n_shots = n_shots;
      s->precision = precision;
      s->n_nodes = (size_t)(nx + 1) * (ny + 1) * (nz + 1);
      s->n_elem = (size_t)nx * ny * nz;
      s->geom = make_geom(nx, ny, nz, s->chunk_planes, 16);
      const Geom& g = s->geom;
      s->u[0].alloc((size_t)n_shots * s->vec());
      s->u[1].alloc((size_t)n_shots * s->vec());
      s->mat.alloc(2 * s->n_elem);
      s->acoef.alloc(s->n_nodes);
      s->step_base.alloc(1);
      upload(s->alane_bf16, make_alane_bf16(OVFEM_ELEMENT_OVFEM), s->stream);
      upload(s->alane_i8, make_alane_i8(OVFEM_ELEMENT_OVFEM), s->stream);
      s->wavelet.alloc(1);
      s->traces.alloc(1);
      s->src = s->build_sources(g, {}, {}, {});
      s->rec = s->build_receivers(g, {});
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
    require(precision != OVFEM_INT8_BF16 || s->stages == 8,
            "ovfem_set_precision: OVFEM_INT8_BF16 runs 8 digit stages only (call ovfem_set_stages(s, 8) first)");
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
    const bool tri = s->element == OVFEM_ELEMENT_TRILINEAR;
    const double sl = kElemScaleLam[tri ? 1 : 0], sm = kElemScaleMu[tri ? 1 : 0];
    std::vector<double> al(576), am(576);
    for (int i = 0; i < 24; ++i)
      for (int j = 0; j < 24; ++j) {
        al[i * 24 + j] = (tri ? kTri.AL[i][j] : kRef.AL[i][j]) / sl;
        am[i * 24 + j] = (tri ? kTri.AM[i][j] : kRef.AM[i][j]) / sm;
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
          mt[2 * e] = h * L / sl;
          mt[2 * e + 1] = h * M / sm;
          const double me = R * h * h * h / 8.0;
          // lambda_max(lam K_lam + mu K_mu) <= max(lam, 0) lambda_max(K_lam) + mu lambda_max(K_mu)
          wmax2 = std::max(wmax2, h * (std::max(L, 0.0) * el + M * em) / me);
          for (int dk = 0; dk < 2; ++dk)
            for (int dj = 0; dj < 2; ++dj)
              for (int di = 0; di < 2; ++di)
                mass[(size_t)((i + di) + (nx + 1) * ((j + dj) + (ny + 1) * (k + dk)))] += me;
        }
    s->wmax2 = wmax2;
    OVFEM_HIP(hipStreamSynchronize(s->stream));  // earlier steps may still read mat
    OVFEM_HIP(hipMemcpyAsync(s->mat.p, mt.data(), 2 * ne * sizeof(double), hipMemcpyHostToDevice, s->stream));
    OVFEM_HIP(hipStreamSynchronize(s->stream));
    s->mass.swap(mass);
    s->model_set = true;
    s->acoef_dirty = true;
    if (s->dt_set && s->dt > s->dt_limit(s->beta)) s->dt_set = false;  // dt must be set again
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
    const double lim = s->dt_limit(s->beta);
    require(dt <= lim, "ovfem_set_dt: dt = " + std::to_string(dt) + " exceeds the element stability bound " +
                           std::to_string(lim) + (s->beta > 0 ? " (with the stiffness-proportional damping)" : ""));
    s->dt = dt;
    s->dt_set = true;
    s->acoef_dirty = true;
    s->invalidate_launches();  // the damping coefficients depend on dt
  });
}

ovfem_status ovfem_set_sources(ovfem_solver* s, int32_t n, const int64_t* node, const int32_t* comp,
                               const int32_t* shot, const double* wavelet, int64_t nt) {
  return guarded([&] {
    require(s != nullptr, "ovfem_set_sources: solver is NULL");
    s->check_device();
    require(n >= 0, "ovfem_set_sources: n < 0");
    require(n == 0 || (node && comp && wavelet && nt > 0), "ovfem_set_sources: missing arrays or nt <= 0");
    require((double)n * (double)std::max<int64_t>(nt, 1) < 2147483647.0, "ovfem_set_sources: table too large");
    std::vector<int64_t> nd(n);
    std::vector<int32_t> cp(n), sh(n);
    for (int i = 0; i < n; ++i) {
      require(node[i] >= 0 && (size_t)node[i] < s->n_nodes, "ovfem_set_sources: node out of range");
      require(comp[i] >= 0 && comp[i] < 3, "ovfem_set_sources: comp out of range");
      require(shot == nullptr || (shot[i] >= 0 && shot[i] < s->n_shots), "ovfem_set_sources: shot out of range");
      nd[i] = node[i];
      cp[i] = comp[i];
      sh[i] = shot ? shot[i] : 0;
    }
    SourceTables st;
    DevBuf<double> dw;
    try {
      st = s->build_sources(s->geom, nd, cp, sh);
      dw.alloc((size_t)n * (size_t)std::max<int64_t>(nt, 1));
      if (n > 0)
        OVFEM_HIP(hipMemcpyAsync(dw.p, wavelet, (size_t)n * nt * sizeof(double), hipMemcpyHostToDevice, s->stream));
      OVFEM_HIP(hipStreamSynchronize(s->stream));
    } catch (...) {
      st.free();
      dw.free();
      throw;
    }
    std::swap(s->src, st);
    std::swap(s->wavelet, dw);
    st.free();
    dw.free();
    s->src_node_h.swap(nd);
    s->src_comp_h.swap(cp);
    s->src_shot_h.swap(sh);
    s->n_src = n;
    s->src_nt = n > 0 ? (int)nt : 0;
    s->invalidate_launches();
  });
}

ovfem_status ovfem_set_receivers(ovfem_solver* s, int32_t n, const int64_t* node, int64_t nt_max) {
  return guarded([&] {
    require(s != nullptr, "ovfem_set_receivers: solver is NULL");
    s->check_device();
    require(n >= 0 && nt_max >= 0, "ovfem_set_receivers: negative count");
    require(n == 0 || node, "ovfem_set_receivers: node is NULL");
    require(nt_max < 2147483647 && (double)n * 3.0 * (double)nt_max < 2147483647.0,
            "ovfem_set_receivers: trace buffer too large");
    std::vector<int64_t> nd(n);
    for (int i = 0; i < n; ++i) {
      require(node[i] >= 0 && (size_t)node[i] < s->n_nodes, "ovfem_set_receivers: node out of range");
      nd[i] = node[i];
    }
    ReceiverTables rt;
    DevBuf<double> tr;
    try {
      rt = s->build_receivers(s->geom, nd);
      tr.alloc((size_t)s->n_shots * n * 3 * nt_max);
      OVFEM_HIP(hipMemsetAsync(tr.p, 0, tr.n * sizeof(double), s->stream));
      OVFEM_HIP(hipStreamSynchronize(s->stream));
    } catch (...) {
      rt.free();
      tr.free();
      throw;
    }
    std::swap(s->rec, rt);
    std::swap(s->traces, tr);
    rt.free();
    tr.free();
    s->rec_node_h.swap(nd);
    s->n_rec = n;
    s->rec_nt = (int)nt_max;
    s->invalidate_launches();
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
    const size_t bytes = s->vec() * sizeof(double);
    const char *a = (const char*)u, *b = (const char*)Ku;
    require(a + bytes <= b || b + bytes <= a, "ovfem_matvec: u and Ku overlap");
    s->check_device();
    KArgs A = s->shot_args(0, s->phase);
    A.u = u;
    A.ku = Ku;
    A.src_nt = 0;
    A.rec_nt = 0;
    launch_unit<MODE_MATVEC>(s->form(), A, nullptr, 0, s->stream);
  });
}

ovfem_status ovfem_get_wavefield(ovfem_solver* s, int32_t which, double* out) {
  return guarded([&] {
    require(s != nullptr, "ovfem_get_wavefield: solver is NULL");
    s->check_device();
    require(which == 0 || which == 1, "ovfem_get_wavefield: which must be 0 or 1");
    require(out != nullptr, "ovfem_get_wavefield: out is NULL");
    const int src = which == 0 ? s->buf_cur(s->phase) : s->buf_prev(s->phase);
    OVFEM_HIP(hipMemcpyAsync(out, s->u[src].p, (size_t)s->n_shots * s->vec() * sizeof(double),
                             hipMemcpyDeviceToDevice, s->stream));
    OVFEM_HIP(hipStreamSynchronize(s->stream));
  });
}

ovfem_status ovfem_set_wavefield(ovfem_solver* s, const double* un, const double* unm1, int64_t step) {
  return guarded([&] {
    require(s != nullptr, "ovfem_set_wavefield: solver is NULL");
    require(un && unm1, "ovfem_set_wavefield: NULL array");
    require(step >= 0, "ovfem_set_wavefield: step < 0");
    s->check_device();
    const size_t bytes = (size_t)s->n_shots * s->vec() * sizeof(double);
    OVFEM_HIP(hipMemcpyAsync(s->u[s->buf_cur(s->phase)].p, un, bytes, hipMemcpyDeviceToDevice, s->stream));
    OVFEM_HIP(hipMemcpyAsync(s->u[s->buf_prev(s->phase)].p, unm1, bytes, hipMemcpyDeviceToDevice, s->stream));
    s->step = step;
    s->ckpt_valid = false;
    OVFEM_HIP(hipStreamSynchronize(s->stream));
  });
}

ovfem_status ovfem_get_traces(ovfem_solver* s, double* out) {
  return guarded([&] {
    require(s != nullptr, "ovfem_get_traces: solver is NULL");
    s->check_device();
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

ovfem_status ovfem_set_element(ovfem_solver* s, int32_t element) {
  return guarded([&] {
    require(s != nullptr, "ovfem_set_element: solver is NULL");
    require(element == OVFEM_ELEMENT_OVFEM || element == OVFEM_ELEMENT_TRILINEAR, "ovfem_set_element: unknown element");
    s->check_device();
    if (element == s->element) return;
    DevBuf<uint32_t> bf;
    DevBuf<uint64_t> i8;
    try {
      upload(bf, make_alane_bf16(element), s->stream);
      upload(i8, make_alane_i8(element), s->stream);
      OVFEM_HIP(hipStreamSynchronize(s->stream));
    } catch (...) {
      bf.free();
      i8.free();
      throw;
    }
    std::swap(s->alane_bf16, bf);
    std::swap(s->alane_i8, i8);
    bf.free();
    i8.free();
    s->element = element;
    s->model_set = false;  // the stored material scaling belongs to the element
    s->dt_set = false;
    s->invalidate_launches();
    s->zero_state();
    OVFEM_HIP(hipStreamSynchronize(s->stream));
  });
}

ovfem_status ovfem_set_damping(ovfem_solver* s, double alpha, double beta) {
  return guarded([&] {
    require(s != nullptr, "ovfem_set_damping: solver is NULL");
    require(std::isfinite(alpha) && std::isfinite(beta) && alpha >= 0.0 && beta >= 0.0,
            "ovfem_set_damping: alpha and beta must be finite and >= 0");
    s->check_device();
    if (s->dt_set)
      require(s->dt <= s->dt_limit(beta), "ovfem_set_damping: dt = " + std::to_string(s->dt) +
                                              " exceeds the stability bound with this beta (" +
                                              std::to_string(s->dt_limit(beta)) + ")");
    if ((alpha != 0.0 || beta != 0.0) && !s->u[2].p) {
      DevBuf<double> u2;
      u2.alloc((size_t)s->n_shots * s->vec());
      std::swap(s->u[2], u2);
    }
    OVFEM_HIP(hipStreamSynchronize(s->stream));
    s->alpha = alpha;
    s->beta = beta;
    s->acoef_dirty = true;
    s->invalidate_launches();
    s->zero_state();
    OVFEM_HIP(hipStreamSynchronize(s->stream));
  });
}

ovfem_status ovfem_set_stages(ovfem_solver* s, int32_t stages) {
  return guarded([&] {
    require(s != nullptr, "ovfem_set_stages: solver is NULL");
    require(stages >= 4 && stages <= 8, "ovfem_set_stages: stages must be in 4..8");
    require(s->precision != OVFEM_INT8_BF16 || stages == 8,
            "ovfem_set_stages: OVFEM_INT8_BF16 runs 8 digit stages only");
    s->stages = stages;
  });
}

ovfem_status ovfem_get_stages(ovfem_solver* s, int32_t* stages) {
  return guarded([&] {
    require(s != nullptr && stages != nullptr, "ovfem_get_stages: NULL argument");
    *stages = s->stages;
  });
}

ovfem_status ovfem_set_tuning(ovfem_solver* s, int32_t chunk_planes, int32_t persistent_groups,
                              int32_t graph_steps) {
  return guarded([&] {
    require(s != nullptr, "ovfem_set_tuning: solver is NULL");
    require(chunk_planes >= 1 && chunk_planes <= 4096, "ovfem_set_tuning: chunk_planes must be in 1..4096");
    require(persistent_groups >= 0, "ovfem_set_tuning: persistent_groups < 0");
    require(graph_steps >= 0 && graph_steps <= 4096 && graph_steps % 2 == 0,
            "ovfem_set_tuning: graph_steps must be even and in 0..4096");
    s->check_device();
    if (make_geom(s->nx, s->ny, s->nz, chunk_planes, s->geom.ty).tz != s->geom.tz)
      s->retile(chunk_planes, s->geom.ty);
    s->chunk_planes = chunk_planes;
    s->persist_groups = persistent_groups;
    s->graph_steps = graph_steps;
    s->invalidate_launches();
  });
}

ovfem_status ovfem_set_tile_rows(ovfem_solver* s, int32_t rows) {
  return guarded([&] {
    require(s != nullptr, "ovfem_set_tile_rows: solver is NULL");
    require(rows == 16 || rows == 32, "ovfem_set_tile_rows: rows must be 16 or 32");
    s->check_device();
    if (rows != s->geom.ty) s->retile(s->chunk_planes, rows);
  });
}

ovfem_status ovfem_get_tile_rows(ovfem_solver* s, int32_t* rows) {
  return guarded([&] {
    require(s != nullptr && rows != nullptr, "ovfem_get_tile_rows: NULL argument");
    *rows = s->geom.ty;
  });
}

ovfem_status ovfem_get_tuning(ovfem_solver* s, int32_t* chunk_planes, int32_t* persistent_groups,
                              int32_t* graph_steps) {
  return guarded([&] {
    require(s != nullptr && chunk_planes && persistent_groups && graph_steps, "ovfem_get_tuning: NULL argument");
    *chunk_planes = s->chunk_planes;
    *persistent_groups = s->persist_groups;
    *graph_steps = s->graph_steps;
  });
}

ovfem_status ovfem_autotune(ovfem_solver* s, int32_t steps, double* best_ms_per_step) {
  return guarded([&] {
    require(s != nullptr, "ovfem_autotune: solver is NULL");
    require(steps >= 2 && steps <= 100000, "ovfem_autotune: steps must be in 2..100000");
    require(s->model_set && s->dt_set, "ovfem_autotune: model and dt not set", OVFEM_ESTATE);
    s->check_device();
    const size_t nv = (size_t)s->n_shots * s->vec(), bytes = nv * sizeof(double);
    DevBuf<double> keep, keep_tr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const int64_t step0 = s->step;
    const int g0 = s->graph_steps;
    int best_planes = s->chunk_planes, best_persist = s->persist_groups, best_rows = s->geom.ty;
    double best = std::numeric_limits<double>::infinity();
    auto cleanup = [&] {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      keep.free();
      keep_tr.free();
    };
    try {
      // the state (wavefield pair, traces, step counter) is saved and restored
      keep.alloc(2 * nv);
      keep_tr.alloc(s->traces.n);
      OVFEM_HIP(hipMemcpyAsync(keep.p, s->u[s->buf_cur(s->phase)].p, bytes, hipMemcpyDeviceToDevice, s->stream));
      OVFEM_HIP(hipMemcpyAsync(keep.p + nv, s->u[s->buf_prev(s->phase)].p, bytes, hipMemcpyDeviceToDevice,
                               s->stream));
      OVFEM_HIP(hipMemcpyAsync(keep_tr.p, s->traces.p, s->traces.n * sizeof(double), hipMemcpyDeviceToDevice,
                               s->stream));
      OVFEM_HIP(hipEventCreate(&e0));
      OVFEM_HIP(hipEventCreate(&e1));
      // time on a filled wavefield pair (restored below)
      const unsigned fill_blocks = (unsigned)((nv + 255) / 256);
      fill_random_kernel<<<fill_blocks, 256, 0, s->stream>>>(s->u[s->buf_cur(s->phase)].p, nv, 1, 1e-6);
      OVFEM_HIP(hipGetLastError());
      fill_random_kernel<<<fill_blocks, 256, 0, s->stream>>>(s->u[s->buf_prev(s->phase)].p, nv, 2, 1e-6);
      OVFEM_HIP(hipGetLastError());
      std::vector<int> plane_opts = {8, 12, 16, 24, 32, 48, 64, 96};
      std::vector<int> persist_opts = {0};
      if (s->n_shots > 1) {
        hipDeviceProp_t prop;
        OVFEM_HIP(hipGetDeviceProperties(&prop, s->device));
        const int cus = std::max(8, prop.multiProcessorCount);
        persist_opts = {0, 2 * cus, 4 * cus};
      }
      s->ckpt_valid = false;
      s->graph_steps = 0;  // plain launches for the tiling and grid choice
      struct Candidate {
        int rows, planes, persist;
        double ms;
      };
      std::vector<Candidate> cands;
      for (int rows : {16, 32}) {
        int last_tz = -1;
        for (int pl : plane_opts) {
          const int tz = make_geom(s->nx, s->ny, s->nz, pl, rows).tz;
          if (tz == last_tz) continue;
          last_tz = tz;
          for (int pg : persist_opts) cands.push_back({rows, pl, pg, std::numeric_limits<double>::infinity()});
        }
      }
      // two passes, each candidate keeping its faster time: the first pass also brings the
      // clocks up, which would otherwise favour whichever candidates run last
      for (int pass = 0; pass < 2; ++pass) {
        for (Candidate& c : cands) {
          if (s->chunk_planes != c.planes || s->geom.ty != c.rows) s->retile(c.planes, c.rows);
          s->persist_groups = c.persist;
          s->invalidate_launches();
          s->do_steps(2);  // warm-up: tables, caches
          OVFEM_HIP(hipEventRecord(e0, s->stream));
          s->do_steps(steps);
          OVFEM_HIP(hipEventRecord(e1, s->stream));
          OVFEM_HIP(hipEventSynchronize(e1));
          float ms = 0;
          OVFEM_HIP(hipEventElapsedTime(&ms, e0, e1));
          c.ms = std::min(c.ms, (double)ms / steps);
        }
      }
      for (const Candidate& c : cands)
        if (c.ms < best) {
          best = c.ms;
          best_planes = c.planes;
          best_persist = c.persist;
          best_rows = c.rows;
        }
      s->retile(best_planes, best_rows);
      s->persist_groups = best_persist;
      // captured blocks against plain launches, at the chosen tiling
      const int64_t gsteps = std::max<int64_t>(64, ((int64_t)steps + 63) / 64 * 64);
      double best_graph = std::numeric_limits<double>::infinity();
      int best_gs = 0;
      for (int gs : {0, 64}) {
        if (gs > 0 && s->damped()) continue;  // damped runs are not captured
        s->graph_steps = gs;
        s->invalidate_launches();
        s->do_steps(gs > 0 ? gs : 2);  // warm-up; captures the block
        OVFEM_HIP(hipEventRecord(e0, s->stream));
        s->do_steps(gsteps);
        OVFEM_HIP(hipEventRecord(e1, s->stream));
        OVFEM_HIP(hipEventSynchronize(e1));
        float ms = 0;
        OVFEM_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms / gsteps < best_graph) {
          best_graph = ms / gsteps;
          best_gs = gs;
        }
      }
      best = std::min(best, best_graph);
      s->graph_steps = best_gs;
      s->invalidate_launches();
      OVFEM_HIP(hipMemcpyAsync(s->u[s->buf_cur(s->phase)].p, keep.p, bytes, hipMemcpyDeviceToDevice, s->stream));
      OVFEM_HIP(hipMemcpyAsync(s->u[s->buf_prev(s->phase)].p, keep.p + nv, bytes, hipMemcpyDeviceToDevice,
                               s->stream));
      OVFEM_HIP(hipMemcpyAsync(s->traces.p, keep_tr.p, s->traces.n * sizeof(double), hipMemcpyDeviceToDevice,
                               s->stream));
      s->step = step0;
      OVFEM_HIP(hipStreamSynchronize(s->stream));
    } catch (...) {
      s->graph_steps = g0;
      (void)hipStreamSynchronize(s->stream);
      cleanup();
      throw;
    }
    cleanup();
    if (best_ms_per_step) *best_ms_per_step = best;
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
      // every = 1: the tape u^{-1} .. u^{max_steps}; otherwise a (u^s, u^{s-1}) pair per slot
      const double vectors = every == 1 ? (double)slots + 1.0 : 2.0 * (double)slots;
      require(vectors * (double)s->n_shots * (double)s->vec() * sizeof(double) < 1e18,
              "ovfem_set_checkpointing: max_steps / every too large for any device", OVFEM_ENOMEM);
      buf.alloc((size_t)(every == 1 ? slots + 1 : slots * 2) * s->n_shots * s->vec());
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
            "then step from reset without changing precision, tiling or wavefield)",
            OVFEM_ESTATE);
    require(n >= 1, "ovfem_adjoint: no forward steps to differentiate", OVFEM_ESTATE);
    require(s->n_rec > 0 && n <= s->rec_nt, "ovfem_adjoint: receivers must record every forward step", OVFEM_ESTATE);
    require(s->model_set && s->dt_set, "ovfem_adjoint: model and dt not set", OVFEM_ESTATE);
    s->refresh_acoef();
    const int64_t every = s->ckpt_every;
    const int shots = s->n_shots;
    const size_t vec = s->vec();
    const size_t all = (size_t)shots * vec;  // the nodal vectors of every shot, [shot][node][3]
    const Geom& g = s->geom;

    // adjoint sources: each receiver component of each shot, driven by its residual row
    // (shot v's tile lists at v (n_wg + 1), as the forward source tables are laid out)
    std::vector<std::vector<int>> per(g.n_wg);
    for (int r = 0; r < s->n_rec; ++r) per[ovfem_solver::tile_of(g, s->rec_node_h[r])].push_back(r);
    std::vector<int> aptr((size_t)shots * (g.n_wg + 1), 0), anode, acomp, arow;
    for (int v = 0; v < shots; ++v) {
      int* ptr = aptr.data() + (size_t)v * (g.n_wg + 1);
      ptr[0] = (int)anode.size();
      for (int w = 0; w < g.n_wg; ++w) {
        for (int r : per[w])
          for (int c = 0; c < 3; ++c) {
            anode.push_back((int)s->rec_node_h[r]);
            acomp.push_back(c);
            arow.push_back(3 * (v * s->n_rec + r) + c);
          }
        ptr[w + 1] = (int)anode.size();
      }
    }
    DevBuf<int> d_aptr, d_anode, d_acomp, d_arow;
    DevBuf<double> seg, wbuf;
    auto free_all = [&] {
      for (auto* b : {&d_aptr, &d_anode, &d_acomp, &d_arow}) b->free();
      seg.free();
      wbuf.free();
    };
    try {
      upload(d_aptr, aptr, s->stream);
      upload(d_anode, anode, s->stream);
      upload(d_acomp, acomp, s->stream);
      upload(d_arow, arow, s->stream);
      seg.alloc((size_t)(every + 1) * all);
      const bool damped = s->damped();
      const double bd = damped ? s->damp_b() : 0.0;
      wbuf.alloc(3 * all);
      OVFEM_HIP(hipMemsetAsync(g_lam, 0, s->n_elem * sizeof(double), s->stream));
      OVFEM_HIP(hipMemsetAsync(g_mu, 0, s->n_elem * sizeof(double), s->stream));
      OVFEM_HIP(hipMemsetAsync(wbuf.p, 0, 3 * all * sizeof(double), s->stream));
      // w[i1] = w^{m+1}, w[i2] = w^{m+2}; a step writes w^m over w^{m+2} (undamped) or
      // into the third buffer (damped: the halo of w^{m+2} is read by neighbours)
      double* w[3] = {wbuf.p, wbuf.p + all, wbuf.p + 2 * all};
      int i1 = 0, i2 = 1;

      // forward recompute: forward sources, no recording; every shot in one launch
      KArgs F = s->shot_args(0, s->phase);
      F.rec_nt = 0;
      F.n_units = shots;
      F.unit_u = (long long)vec;
      F.unit_src = g.n_wg + 1;
      F.unit_tr = 0;
      KArgs B = F;  // adjoint steps: the residual injected at the receivers
      B.src_ptr = d_aptr.p;
      B.src_node = d_anode.p;
      B.src_comp = d_acomp.p;
      B.src_row = d_arow.p;
      B.wavelet = residual;
      B.src_nt = s->rec_nt;
      // gradient terms: 16 x 16-element tiles by chunks of zc element layers (at least 4,
      // so that a chunk's extra staged plane costs at most a quarter; deeper while the grid
      // still has 2048 work-groups)
      const int gtiles = ((int)s->nx + GT - 1) / GT * (((int)s->ny + GT - 1) / GT);
      const int zc = (int)std::max<int64_t>(4, std::min<int64_t>(16, (int64_t)gtiles * s->nz / 2048));
      const int gblocks = gtiles * (int)((s->nz + zc - 1) / zc);
      // one launch per shot, in shot order: each element's sums run over the shots in turn
      auto gradient = [&](const double* u1, const double* u2, const double* wm) {
        const bool tri = s->element == OVFEM_ELEMENT_TRILINEAR;
        if (u2 && tri)
          ovfem_gradient_kernel<1, true><<<gblocks, GT * GT, 0, s->stream>>>(g, zc, s->h, s->mat.p, u1, u2, bd, wm,
                                                                             g_lam, g_mu);
        else if (u2)
          ovfem_gradient_kernel<0, true><<<gblocks, GT * GT, 0, s->stream>>>(g, zc, s->h, s->mat.p, u1, u2, bd, wm,
                                                                             g_lam, g_mu);
        else if (tri)
          ovfem_gradient_kernel<1, false><<<gblocks, GT * GT, 0, s->stream>>>(g, zc, s->h, s->mat.p, u1, nullptr, bd,
                                                                              wm, g_lam, g_mu);
        else
          ovfem_gradient_kernel<0, false><<<gblocks, GT * GT, 0, s->stream>>>(g, zc, s->h, s->mat.p, u1, nullptr, bd,
                                                                              wm, g_lam, g_mu);
        OVFEM_HIP(hipGetLastError());
      };

      for (int64_t sg = (n - 1) / every; sg >= 0; --sg) {
        const int64_t s0 = sg * every, e0 = std::min(s0 + every, n);
        // state(k) = u^{s0+k}: u^{s0} and u^{s0-1} from the checkpoint, the rest recomputed.
        // The adjoint steps m = e0 .. s0+1 read u^{m-1} (and u^{m-2} when damped), so the
        // segment needs u^{s0-1} .. u^{e0-1}: e0 - s0 - 1 recomputed steps (none when every
        // step is checkpointed)
        auto state = [&](int64_t k) -> double* {
          if (k < 0) return s->ckpt_u(sg, 1);
          if (k == 0) return s->ckpt_u(sg, 0);
          return seg.p + (size_t)k * all;
        };
        for (int64_t t = s0; t + 1 < e0; ++t) {
          F.u = state(t - s0);
          F.uprev = state(t - s0 - 1);
          F.unext = state(t - s0 + 1);
          launch_unit<MODE_STEP>(s->form(), F, nullptr, t, s->stream);
        }
        for (int64_t m = e0; m > s0; --m) {
          const int inew = damped ? 3 - i1 - i2 : i2;
          B.u = w[i1];
          B.uprev = w[i2];
          B.unext = w[inew];
          launch_unit<MODE_STEP>(s->form(), B, nullptr, m - 1, s->stream);
          i2 = i1;
          i1 = inew;
          for (int v = 0; v < shots; ++v)
            gradient(state(m - 1 - s0) + v * vec, damped ? state(m - 2 - s0) + v * vec : nullptr,
                     w[i1] + v * vec);
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

ovfem_status ovfem_batch_create(ovfem_batch** out, ovfem_solver* const* members, int32_t n) {
  return guarded([&] {
    require(out != nullptr, "ovfem_batch_create: out is NULL");
    *out = nullptr;
    require(members != nullptr && n >= 1 && n <= OVFEM_MAX_BATCH, "ovfem_batch_create: member count out of range");
    for (int i = 0; i < n; ++i) {
      require(members[i] != nullptr, "ovfem_batch_create: NULL member");
      require(members[i]->device == members[0]->device, "ovfem_batch_create: members on different devices");
      require(members[i]->stream == members[0]->stream, "ovfem_batch_create: members on different streams");
      for (int j = 0; j < i; ++j) require(members[j] != members[i], "ovfem_batch_create: repeated member");
    }
    auto b = new ovfem_batch();
    b->members.assign(members, members + n);
    b->stream = members[0]->stream;
    *out = b;
  });
}

ovfem_status ovfem_batch_destroy(ovfem_batch* b) {
  return guarded([&] { delete b; });
}

ovfem_status ovfem_batch_set_tuning(ovfem_batch* b, int32_t persistent_groups) {
  return guarded([&] {
    require(b != nullptr, "ovfem_batch_set_tuning: batch is NULL");
    require(persistent_groups >= 0, "ovfem_batch_set_tuning: persistent_groups < 0");
    b->persist_groups = persistent_groups;
  });
}

ovfem_status ovfem_batch_set_graph(ovfem_batch* b, int32_t graph_steps) {
  return guarded([&] {
    require(b != nullptr, "ovfem_batch_set_graph: batch is NULL");
    require(graph_steps >= 0 && graph_steps % kBatchTables == 0 && graph_steps <= 4096,
            "ovfem_batch_set_graph: graph_steps must be a multiple of 6 in 0..4096");
    OVFEM_HIP(hipStreamSynchronize(b->stream));
    b->drop_graph();
    b->graph_steps = graph_steps;
  });
}

ovfem_status ovfem_batch_step(ovfem_batch* b, int64_t n) {
  return guarded([&] {
    require(b != nullptr, "ovfem_batch_step: batch is NULL");
    require(n >= 0, "ovfem_batch_step: n < 0");
    b->check_members();
    if (n == 0) return;
    for (auto* m : b->members) m->prepare_steps();
    std::vector<KArgs> t;
    std::vector<int> bg;
    b->tables(t, bg);
    const bool same = t.size() == b->t_host.size() && bg == b->begin_host &&
                      std::memcmp(t.data(), b->t_host.data(), t.size() * sizeof(KArgs)) == 0;
    if (!same) {
      if (b->units.n < t.size() || b->begin.n < bg.size()) {
        OVFEM_HIP(hipStreamSynchronize(b->stream));  // earlier launches may still read the old tables
        b->drop_graph();
        b->units.alloc(t.size());
        b->begin.alloc(bg.size());
      }
      b->t_host.swap(t);
      b->begin_host.swap(bg);
      // stream-ordered after the launches that read the previous contents
      OVFEM_HIP(hipMemcpyAsync(b->units.p, b->t_host.data(), b->t_host.size() * sizeof(KArgs),
                               hipMemcpyHostToDevice, b->stream));
      OVFEM_HIP(hipMemcpyAsync(b->begin.p, b->begin_host.data(), b->begin_host.size() * sizeof(int),
                               hipMemcpyHostToDevice, b->stream));
    }
    b->launch(b->units.p, b->begin.p, b->begin_host, n, true);
  });
}

ovfem_status ovfem_batch_step_noalloc(ovfem_batch* b, int64_t n) {
  return guarded([&] {
    require(b != nullptr, "ovfem_batch_step_noalloc: batch is NULL");
    require(n >= 0, "ovfem_batch_step_noalloc: n < 0");
    b->check_members();
    for (size_t i = 0; i < b->members.size(); ++i) {
      const ovfem_solver* m = b->members[i];
      require(m->model_set && m->dt_set, "ovfem_batch_step_noalloc: member " + std::to_string(i) +
                                             " has no model or dt", OVFEM_ESTATE);
      require(!m->acoef_dirty, "ovfem_batch_step_noalloc: member " + std::to_string(i) +
                                   " changed since it last stepped; step it once (ovfem_step with n = 0) to "
                                   "build its tables",
              OVFEM_ESTATE);
    }
    if (n == 0) return;
    b->tables(b->t_fixed, b->begin_fixed);
    const size_t tb = b->t_fixed.size() * sizeof(KArgs), bb = b->begin_fixed.size() * sizeof(int);
    require(tb + bb <= OVFEM_NOALLOC_SCRATCH_BYTES,
            "ovfem_batch_step_noalloc: the batch's argument tables take " + std::to_string(tb + bb) +
                " bytes (" + std::to_string(b->begin_fixed.size() - 1) + " units); the fixed array holds " +
                std::to_string((size_t)OVFEM_NOALLOC_SCRATCH_BYTES));
    unsigned char* p = scratch_address();
    // stream-ordered after every earlier use of the array on this stream
    OVFEM_HIP(hipMemcpyAsync(p, b->t_fixed.data(), tb, hipMemcpyHostToDevice, b->stream));
    OVFEM_HIP(hipMemcpyAsync(p + tb, b->begin_fixed.data(), bb, hipMemcpyHostToDevice, b->stream));
    b->launch(reinterpret_cast<const KArgs*>(p), reinterpret_cast<const int*>(p + tb), b->begin_fixed, n, false);
  });
}

ovfem_status ovfem_check_finite(ovfem_solver* s, int32_t* finite) {
  return guarded([&] {
    require(s != nullptr && finite != nullptr, "ovfem_check_finite: NULL argument");
    s->check_device();
    const size_t nv = (size_t)s->n_shots * s->vec();
    DevBuf<int> flags;
    flags.alloc(2 * kFiniteBlocks);
    nonfinite_kernel<<<kFiniteBlocks, 256, 0, s->stream>>>(s->u[s->buf_cur(s->phase)].p, nv, flags.p);
    OVFEM_HIP(hipGetLastError());
    nonfinite_kernel<<<kFiniteBlocks, 256, 0, s->stream>>>(s->u[s->buf_prev(s->phase)].p, nv, flags.p + kFiniteBlocks);
    OVFEM_HIP(hipGetLastError());
    std::vector<int> h(2 * kFiniteBlocks);
    OVFEM_HIP(hipMemcpyAsync(h.data(), flags.p, h.size() * sizeof(int), hipMemcpyDeviceToHost, s->stream));
    OVFEM_HIP(hipStreamSynchronize(s->stream));
    int bad = 0;
    for (int f : h) bad |= f;
    *finite = bad ? 0 : 1;
  });
}

ovfem_status ovfem_synchronize(ovfem_solver* s) {
  return guarded([&] {
    require(s != nullptr, "ovfem_synchronize: solver is NULL");
    OVFEM_HIP(hipStreamSynchronize(s->stream));
  });
}

}  // extern "C"
