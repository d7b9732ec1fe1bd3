// Host side of the C ABI declared in include/sw.h: validation, quadtree faces,
// reference tables, device memory, and the per-step launch sequence.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "sw.h"
#include "sw_internal.h"

namespace swk {
hipError_t launch_stage_r1(int P, int mode, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_stage_r2(int P, int mode, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_stage_r3(int P, int mode, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_stage_scan_r1(int P, int mode, int mode2, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_stage_scan_r2(int P, int mode, int mode2, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_stage_scan_r3(int P, int mode, int mode2, const StageArgs& a, int nblk, hipStream_t s);

hipError_t launch_stage_scan(int r, int P, int mode, int mode2, const StageArgs& a, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  switch (r) {
    case 1: return launch_stage_scan_r1(P, mode, mode2, a, nblk, s);
    case 2: return launch_stage_scan_r2(P, mode, mode2, a, nblk, s);
    case 3: return launch_stage_scan_r3(P, mode, mode2, a, nblk, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_stage(int r, int P, int mode, const StageArgs& a, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  switch (r) {
    case 1: return launch_stage_r1(P, mode, a, nblk, s);
    case 2: return launch_stage_r2(P, mode, a, nblk, s);
    case 3: return launch_stage_r3(P, mode, a, nblk, s);
  }
  return hipErrorInvalidValue;
}

__global__ void k_bathy(const double*, const double*, double*, int, int, int, size_t);
__global__ void k_facez(const int*, const int*, const int*, int, int, int, int, int, size_t, const double*,
                        const double*, const double*, double*, int*, int);
__global__ void k_cellinit(LevelTabs, int, int, size_t, int, const double*, const double*, double*, double*);
__global__ void k_lake(LevelTabs, int, int, size_t, int, const double*, const double*, const double*, double*,
                       double*, double*);
__global__ void k_fill(double*, size_t, double);
__global__ void k_fill8(int8_t*, size_t, int8_t);
__global__ void k_copy(const double*, double*, size_t);
__global__ void k_fill_n(double*, int, double);
__global__ void k_copy8(const int8_t*, int8_t*, size_t);
__global__ void k_minred_seg(const double*, const int*, double*);
__global__ void k_dt_seg(const double*, const int*, const double*, double*);
__global__ void k_min_all(const double*, int, double*);
__global__ void k_diag_part_seg(const double*, const int8_t*, const int*, double*);
__global__ void k_diag_seg(const double*, const int*, double*, double*, const double*);

hipError_t launch_elem_r1(int P, int mode, int wpb, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_elem_r2(int P, int mode, int wpb, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_elem_r3(int P, int mode, int wpb, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_vjp_vol_r1(int P, int mode, const VjpArgs& a, int nblk, hipStream_t s);
hipError_t launch_vjp_vol_r2(int P, int mode, const VjpArgs& a, int nblk, hipStream_t s);
hipError_t launch_vjp_vol_r3(int P, int mode, const VjpArgs& a, int nblk, hipStream_t s);
__global__ void k_gather_fdb(const double*, const int*, const int*, int, double*);
__global__ void k_vjp_combine(double*, double*, double*, const double*, int, size_t);

hipError_t launch_vjp_vol(int r, int P, int mode, const VjpArgs& a, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  switch (r) {
    case 1: return launch_vjp_vol_r1(P, mode, a, nblk, s);
    case 2: return launch_vjp_vol_r2(P, mode, a, nblk, s);
    case 3: return launch_vjp_vol_r3(P, mode, a, nblk, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_elem(int r, int P, int mode, int wpb, const StageArgs& a, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  switch (r) {
    case 1: return launch_elem_r1(P, mode, wpb, a, nblk, s);
    case 2: return launch_elem_r2(P, mode, wpb, a, nblk, s);
    case 3: return launch_elem_r3(P, mode, wpb, a, nblk, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_trc_r1(int P, int mode, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_trc_r2(int P, int mode, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_trc_r3(int P, int mode, const StageArgs& a, int nblk, hipStream_t s);

hipError_t launch_trc(int r, int P, int mode, const StageArgs& a, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  switch (r) {
    case 1: return launch_trc_r1(P, mode, a, nblk, s);
    case 2: return launch_trc_r2(P, mode, a, nblk, s);
    case 3: return launch_trc_r3(P, mode, a, nblk, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_trc_degree_r1(int P, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_trc_degree_r2(int P, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_trc_degree_r3(int P, const StageArgs& a, int nblk, hipStream_t s);

hipError_t launch_trc_degree(int r, int P, const StageArgs& a, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  switch (r) {
    case 1: return launch_trc_degree_r1(P, a, nblk, s);
    case 2: return launch_trc_degree_r2(P, a, nblk, s);
    case 3: return launch_trc_degree_r3(P, a, nblk, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_trc_multi_r1(int P, int mode, const StageArgs& a, const TrcSet& ts, int nblk, hipStream_t s);
hipError_t launch_trc_multi_r2(int P, int mode, const StageArgs& a, const TrcSet& ts, int nblk, hipStream_t s);
hipError_t launch_trc_multi_r3(int P, int mode, const StageArgs& a, const TrcSet& ts, int nblk, hipStream_t s);

hipError_t launch_trc_multi(int r, int P, int mode, const StageArgs& a, const TrcSet& ts, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  if (ts.M < 1 || ts.M > kMaxReact) return hipErrorInvalidValue;
  switch (r) {
    case 1: return launch_trc_multi_r1(P, mode, a, ts, nblk, s);
    case 2: return launch_trc_multi_r2(P, mode, a, ts, nblk, s);
    case 3: return launch_trc_multi_r3(P, mode, a, ts, nblk, s);
  }
  return hipErrorInvalidValue;
}
}  // namespace swk

using namespace swk;

namespace {

thread_local std::string g_err;

sw_status fail(sw_status s, const std::string& m) {
  g_err = m;
  return s;
}

#define HIPCHK(x)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) return fail(SW_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// 1-D reference data: Legendre polynomials, GLL / GL / equispaced rules on [0,1],
// Lagrange basis on the GLL support points (Sec. 3.2).
// ---------------------------------------------------------------------------
void legendre(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    p = 1.0;
    dp = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = (std::fabs(x) < 1.0) ? n * (x * p1 - p0) / (x * x - 1.0) : 0.5 * n * (n + 1.0) * (x > 0 ? 1.0 : (n % 2 ? 1.0 : -1.0));
}

// n-point Lobatto rule: end points and the roots of P'_{n-1}, weights 2/(N(N+1)P_N^2)
void gll(int n, std::vector<double>& x, std::vector<double>& w) {
  const int N = n - 1;
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  std::vector<double> t(n);
  t[0] = -1.0;
  t[N] = 1.0;
  for (int i = 1; i < N; ++i) {
    double xi = -std::cos(M_PI * i / N);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(N, xi, p, dp);
      const double d2 = (2.0 * xi * dp - N * (N + 1.0) * p) / (1.0 - xi * xi);
      const double dx = dp / d2;
      xi -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    t[i] = xi;
  }
  for (int i = 0; i < n; ++i) {
    double p, dp;
    legendre(N, t[i], p, dp);
    x[i] = (t[i] + 1.0) * 0.5;
    w[i] = 1.0 / (N * (N + 1.0) * p * p);   // 2/(N(N+1)P^2) halved for [0,1]
  }
  x[0] = 0.0;
  x[N] = 1.0;
}

void gl(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double xi = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(n, xi, p, dp);
      const double dx = p / dp;
      xi -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    double p, dp;
    legendre(n, xi, p, dp);
    x[i] = (xi + 1.0) * 0.5;
    w[i] = 1.0 / ((1.0 - xi * xi) * dp * dp);
  }
}

void eqr(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.assign(n, 1.0 / (n - 1));
  for (int i = 0; i < n; ++i) x[i] = (double)i / (n - 1);
  w[0] = w[n - 1] = 0.5 / (n - 1);
}

double lag(const std::vector<double>& xi, int j, double x) {
  double v = 1.0;
  for (size_t m = 0; m < xi.size(); ++m)
    if ((int)m != j) v *= (x - xi[m]) / (xi[j] - xi[m]);
  return v;
}

double dlag(const std::vector<double>& xi, int j, double x) {
  double s = 0.0;
  for (size_t k = 0; k < xi.size(); ++k) {
    if ((int)k == j) continue;
    double v = 1.0 / (xi[j] - xi[k]);
    for (size_t m = 0; m < xi.size(); ++m)
      if ((int)m != j && m != k) v *= (x - xi[m]) / (xi[j] - xi[m]);
    s += v;
  }
  return s;
}

// In-place inverse of an SPD matrix via Cholesky (n <= 16).
bool spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> L(n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    if (!(s > 0.0)) return false;
    L[j * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / L[j * n + j];
    }
  }
  std::vector<double> inv(n * n, 0.0), e(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= L[i * n + k] * e[k];
      e[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = e[i];
      for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * e[k];
      e[i] = s / L[i * n + i];
    }
    for (int i = 0; i < n; ++i) inv[i * n + c] = e[i];
  }
  A = inv;
  return true;
}

struct LevelH {
  int L = 0, S = 0, P = 0;
  double w1 = 0;
  int cell0 = 0, ncell = 0;
  size_t off = 0;          // offset of this level's samples in the node arrays
  int face0 = 0, nface = 0;  // all faces whose fine (or equal) side is on this level
  size_t zfoff = 0;          // offset of this level's faces in the face-sample array
  // face classes: direction (x: W/E, y: S/N) x (conforming or boundary, sub-face 0,
  // sub-face 1); the faces of one class touch disjoint (cell, dof) sets
  int cface0[6]{}, cnface[6]{}, cfnblk[6]{};
  int nblk = 0;              // general element-kernel blocks (one wavefront each)
  int wpb = 1;               // wavefronts per workgroup of the fast element kernel
  int face_q = kFaceLanes;   // lanes per face of the face kernel
  int xorder = -1;           // fast-kernel cell order over the XCDs: 0 round robin, 1 contiguous,
                             // -1 by the mesh (contiguous on single-level meshes)
  int8_t* d_wflag = nullptr;  // per wavefront (nblk): cells left to the general kernel
  std::vector<double> xh, wh;
  double* d_tab = nullptr;
  LevelTabs tabs{};
  // volume terms on Table 1's Gauss-Legendre rule (SW_QUAD_PAPER): its nodes,
  // weights and tables, and the offset of the level's volume-rule samples
  std::vector<double> xv, wv;
  double* d_vtab = nullptr;
  LevelTabs vtabs{};
  size_t voff = 0;
  double* d_xh = nullptr;    // [S] sample-node positions on [0, 1]
  double* d_xv = nullptr;    // [nv] volume-rule node positions (SW_QUAD_PAPER)
};

// Device memory of contexts is recycled: a context hands its blocks to a
// per-device cache when it is destroyed (its stream synchronised first), and
// later contexts of that device take blocks from it before calling hipMalloc.
// A remesh replaces a context by one of nearly the same size, so it then
// allocates nothing.  Block sizes are rounded up to a multiple of 1/8 of
// their power of two; the cache holds at most kCacheCap bytes per device.
constexpr int kCacheDevices = 64;
constexpr size_t kCacheCap = (size_t)4 << 30;
std::mutex g_cache_mu;
std::unordered_map<size_t, std::vector<void*>> g_cache[kCacheDevices];
size_t g_cache_bytes[kCacheDevices] = {};

size_t block_bytes(size_t n) {
  if (n <= 256) return 256;
  int e = 0;
  while (((size_t)1 << e) < n) ++e;
  const size_t q = (size_t)1 << (e > 3 ? e - 3 : 0);
  return (n + q - 1) / q * q;
}

hipError_t cache_alloc(int dev, size_t bytes, void** p) {
  if (dev >= 0 && dev < kCacheDevices) {
    std::lock_guard<std::mutex> g(g_cache_mu);
    auto it = g_cache[dev].find(bytes);
    if (it != g_cache[dev].end() && !it->second.empty()) {
      *p = it->second.back();
      it->second.pop_back();
      g_cache_bytes[dev] -= bytes;
      return hipSuccess;
    }
  }
  return hipMalloc(p, bytes);
}

// Host-to-device uploads of context set-up: the data are gathered into a
// host blob, copied once into a pinned per-device staging buffer (held for
// the process, guarded by a mutex until the copies have completed) and sent
// with asynchronous copies on one stream.
std::mutex g_stage_mu;
void* g_stage[64] = {};
size_t g_stage_bytes[64] = {};

struct Uploads {
  std::vector<char> blob;
  std::vector<std::pair<void*, std::pair<size_t, size_t>>> item;   // dst, (offset, bytes)
  void add(void* dst, const void* src, size_t bytes) {
    const size_t off = (blob.size() + 255) / 256 * 256;
    blob.resize(off + bytes);
    if (bytes) std::memcpy(blob.data() + off, src, bytes);
    item.push_back({dst, {off, bytes}});
  }
  // issues the copies and waits for them (the staging buffer is shared)
  hipError_t flush(int dev, hipStream_t s) {
    if (item.empty()) return hipSuccess;
    std::lock_guard<std::mutex> g(g_stage_mu);
    const int d = dev >= 0 && dev < 64 ? dev : 0;
    if (g_stage_bytes[d] < blob.size()) {
      if (g_stage[d]) (void)hipHostFree(g_stage[d]);
      g_stage[d] = nullptr;
      g_stage_bytes[d] = 0;
      hipError_t e = hipHostMalloc(&g_stage[d], blob.size(), hipHostMallocDefault);
      if (e != hipSuccess) return e;
      g_stage_bytes[d] = blob.size();
    }
    std::memcpy(g_stage[d], blob.data(), blob.size());
    for (auto& it : item) {
      if (!it.second.second) continue;
      hipError_t e = hipMemcpyAsync(it.first, (char*)g_stage[d] + it.second.first, it.second.second,
                                    hipMemcpyHostToDevice, s);
      if (e != hipSuccess) return e;
    }
    return hipStreamSynchronize(s);
  }
};

void cache_free(int dev, void* p, size_t bytes) {
  if (dev >= 0 && dev < kCacheDevices) {
    std::lock_guard<std::mutex> g(g_cache_mu);
    if (g_cache_bytes[dev] + bytes <= kCacheCap) {
      g_cache[dev][bytes].push_back(p);
      g_cache_bytes[dev] += bytes;
      return;
    }
  }
  (void)hipFree(p);
}

}  // namespace

struct sw_ctx {
  int dev = 0;
  hipStream_t s = nullptr;
  sw_params p{};
  int r = 1, N1 = 2, NP = 4, K = 0, F = 0, ns = 3, M = 1;
  int64_t nvol = 0;          // sample nodes (sum over cells of S^2)
  int nv = 0;                 // SW_QUAD_PAPER: volume-rule nodes per direction (0: the sample rule)
  int64_t nvv = 0;            // volume-rule nodes (K nv^2), stored after the sample nodes
  // members: coarse-grid origin and cell size; per cell: member, index in the
  // member's description, level, integer position, size
  std::vector<double> mx0, my0, mdx0;
  std::vector<int> mnx0, mny0;
  std::vector<std::array<int, 4>> mbc;
  std::vector<int> cmem, cloc, lev, ci, cj;
  std::vector<double> cdx;
  std::vector<LevelH> lv;
  double A[4][4]{}, b[4]{}, c[4]{};
  double At[4][4]{};          // implicit companion (IMEX), zero otherwise
  bool imex = false;
  double* d_lres = nullptr;   // IMEX: implicit-part residuals [slot][2][K][NP]
  double* d_gam = nullptr;    // IMEX: friction matrix of the last volume pass [K][NP(NP+1)/2]
  int *d_fA = nullptr, *d_fB = nullptr, *d_meta = nullptr, *d_err = nullptr, *d_cmem = nullptr;
  int *d_ci = nullptr, *d_cj = nullptr;   // [K] integer cell positions
  double* d_mxy = nullptr;                // [2][M] member origins
  // bathymetry raster (sw_set_bed_grid): bed elevation g[j][i] at
  // (gx0 + i gdx, gy0 + j gdy); sampled at the nodes of new cells by sw_remesh
  double* d_grid = nullptr;
  int gnx = 0, gny = 0;
  double gx0 = 0, gy0 = 0, gdx = 0, gdy = 0;
  double *d_zb = nullptr, *d_braw = nullptr, *d_db = nullptr, *d_bvec = nullptr, *d_zmax = nullptr;
  double *d_nman = nullptr, *d_cdx = nullptr, *d_cw1 = nullptr, *d_zf = nullptr;
  double *d_sn[4]{}, *d_ss[4]{};
  double *d_hn = nullptr, *d_cn = nullptr, *d_res = nullptr, *d_cdiag = nullptr;
  // per member: time, time step, time for sw_apply_operator, tide, CFL number,
  // diagnostics [M][kMDiag], scratch
  double *d_mt = nullptr, *d_mdt = nullptr, *d_mt_apply = nullptr, *d_mtide = nullptr, *d_mcfl = nullptr;
  double *d_mdiag = nullptr, *d_mtmp = nullptr;
  // segmented reductions: face chunks and cell chunks, grouped by member
  double *d_fdt = nullptr, *d_part = nullptr;
  int *d_fch = nullptr, *d_fch_m0 = nullptr, *d_cch = nullptr, *d_cch_m0 = nullptr;
  int nfch = 0, ncch = 0;
  int8_t *d_flag = nullptr, *d_allwet = nullptr, *d_need = nullptr, *d_oflag = nullptr;
  // adjoint: per-face bed-offset parts [F][2] and, per cell, the list of its
  // entries in that array (CSR, face order)
  double* d_fdb = nullptr;
  // given boundary data (state and discharge sides): per face the offset of its
  // nodes in the [4][ng] array (-1: none), faces carrying data in face order
  int* d_gof = nullptr;
  double* d_ghost = nullptr;
  int64_t ng = 0;
  std::vector<int> gface;
  std::vector<int> gcell, gside;   // cell (fine or equal side) and side of each of those faces
  bool ghost_set = false;
  int *d_cfoff = nullptr, *d_cfent = nullptr;
  bool start_ready = false;   // H^n, stage-1 volume terms and degrees of the current state are in place
  // the prepared start came from a tracer replay's final kernel, which left
  // the flow's volume terms out (a coupled step prepares it again)
  bool start_replay = false;
  bool replaying = false;     // inside a tracer replay (sw_tracer_step, sw_step_tracers_react)
  const double* rp[3] = {nullptr, nullptr, nullptr};   // tracer replay: recorded flow of the current stage
  double* d_trec = nullptr;   // sw_step_tracers: the flow record of one step ([ns][3][KN] stages, [3][KN] end)
  hipEvent_t ev_rec = nullptr;  // sw_step_tracers: the record is complete / the tracers are done with it
  double* rec[3] = {nullptr, nullptr, nullptr};        // record of the final combination's flow
  bool fixed_dt = false;
  bool bathy_set = false;
  int stage_done = 0;      // stages completed in the current step (0: no step open)
  int64_t nstep = 0;
  std::vector<std::pair<void*, size_t>> allocs;   // device blocks and their sizes
  // kernel timing (sw_profile): events recorded around each launch group
  bool prof = false;
  int prof_mask = 0xFF;      // kernel classes timed while profiling
  struct Ev { int kind; int nlaunch; hipEvent_t a, b; };
  std::vector<Ev> ev;
  double prof_ms[8]{};
  int64_t prof_n[8]{};

  template <class T>
  sw_status alloc(T** p, size_t n) {
    void* q = nullptr;
    if (n == 0) n = 1;
    const size_t bytes = block_bytes(n * sizeof(T));
    hipError_t e = cache_alloc(dev, bytes, &q);
    if (e != hipSuccess) return fail(SW_ENOMEM, "hipMalloc failed for " + std::to_string(bytes) + " bytes");
    allocs.push_back({q, bytes});
    *p = (T*)q;
    return SW_OK;
  }
  sw_ctx() = default;
  sw_ctx(const sw_ctx&) = delete;
  sw_ctx& operator=(const sw_ctx&) = default;
  void release() {
    if (ev_rec) {
      (void)hipEventDestroy(ev_rec);
      ev_rec = nullptr;
    }
    for (auto& e : ev) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    ev.clear();
    if (!allocs.empty()) (void)hipStreamSynchronize(s);
    for (auto& a : allocs) cache_free(dev, a.first, a.second);
    allocs.clear();
  }
  // Releases this context's device memory and events and takes over n's
  // contents (sw_remesh swaps in the context of the new mesh this way, so the
  // caller's handle stays valid); n is left owning nothing.
  void adopt(sw_ctx& n) {
    release();
    *this = n;
    n.allocs.clear();
    n.ev.clear();
    n.ev_rec = nullptr;
  }
  ~sw_ctx() { release(); }
  // bracket a group of launches of one kernel class with events when profiling
  struct Scope {
    sw_ctx* c;
    int kind, n;
    hipEvent_t a{}, b{};
    bool on = false;
    Scope(sw_ctx* c_, int k, int n_) : c(c_), kind(k), n(n_) {
      if (!c->prof || !((c->prof_mask >> kind) & 1)) return;
      // timing-only events: no system-scope fence (cache write-back) at record,
      // so the measurement does not perturb the launches it brackets
      const unsigned fl = hipEventDisableSystemFence;
      if (hipEventCreateWithFlags(&a, fl) != hipSuccess) return;
      if (hipEventCreateWithFlags(&b, fl) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
      }
      on = hipEventRecord(a, c->s) == hipSuccess;
    }
    ~Scope() {
      if (!on) return;
      (void)hipEventRecord(b, c->s);
      c->ev.push_back({kind, n, a, b});
    }
  };
};

namespace {

constexpr int kNSlot = 5;   // residual slots: up to 4 stages + one for sw_apply_operator
constexpr int kApplySlot = 4;
constexpr int kMDiag = 16;  // per-member diagnostics: D_* slots, [7] dt, [8] t
constexpr int kFaceChunk = 1024, kCellChunk = 256;
constexpr int kListGrid = 1024;   // workgroups of the general kernel walking the wavefront flags

void tableau(int rk, int& s, double A[4][4], double b[4], double c[4]) {
  for (int i = 0; i < 4; ++i) {
    b[i] = c[i] = 0.0;
    for (int j = 0; j < 4; ++j) A[i][j] = 0.0;
  }
  if (rk == SW_RK_FE) {
    s = 1;
    b[0] = 1.0;
  } else if (rk == SW_RK_SSP3) {
    s = 3;
    A[1][0] = 1.0;
    A[2][0] = 0.25;
    A[2][1] = 0.25;
    b[0] = 1.0 / 6.0;
    b[1] = 1.0 / 6.0;
    b[2] = 2.0 / 3.0;
    c[1] = 1.0;
    c[2] = 0.5;
  } else if (rk == SW_RK_RK32 || rk == SW_RK_IMEX) {
    s = 3;
    const double chi = 1.0 - std::sqrt(2.0) / 2.0, a32 = 0.5;
    A[1][0] = 2.0 * chi;
    A[2][0] = 1.0 - a32;
    A[2][1] = a32;
    const double b2 = (1.0 - 2.0 * chi) / (4.0 * chi);
    b[0] = 1.0 - b2 - chi;
    b[1] = b2;
    b[2] = chi;
    c[1] = 2.0 * chi;
    c[2] = 1.0;
  } else {
    s = 4;
    A[1][0] = 0.5;
    A[2][1] = 0.5;
    A[3][2] = 1.0;
    b[0] = 1.0 / 6.0;
    b[1] = 2.0 / 6.0;
    b[2] = 2.0 / 6.0;
    b[3] = 1.0 / 6.0;
    c[1] = 0.5;
    c[2] = 0.5;
    c[3] = 1.0;
  }
}

// implicit (DIRK) companion of the IMEX pair: TR-BDF2, chi = 1 - sqrt(2)/2,
// b~ = b (Appendix A); zero for the explicit schemes
void implicit_tableau(int rk, double At[4][4]) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) At[i][j] = 0.0;
  if (rk != SW_RK_IMEX) return;
  const double chi = 1.0 - std::sqrt(2.0) / 2.0, b2 = (1.0 - 2.0 * chi) / (4.0 * chi);
  At[1][0] = chi;
  At[1][1] = chi;
  At[2][0] = 1.0 - b2 - chi;
  At[2][1] = b2;
  At[2][2] = chi;
}

int64_t key(int L, int i, int j) { return ((int64_t)L << 52) | ((int64_t)i << 26) | (int64_t)j; }

// Cell lookup by (level, i, j): dense arrays for the levels below ndense
// while their grids are small, a hash map for the other levels.  Values: a
// cell index (>= 0) or another code of the caller's (<= -2); -1: none.
class LeafIndex {
 public:
  LeafIndex(int nx0, int ny0, int nlev, int ndense) : nx0_(nx0), ny0_(ny0), nlev_(nlev) {
    int64_t tot = 0;
    ndense = std::min(ndense, nlev);
    for (int L = 0; L < ndense; ++L) tot += ((int64_t)nx0 << L) * ((int64_t)ny0 << L);
    ndense_ = tot <= ((int64_t)1 << 22) ? ndense : 0;
    off_.assign(ndense_ + 1, 0);
    for (int L = 0; L < ndense_; ++L) off_[L + 1] = off_[L] + ((int64_t)nx0 << L) * ((int64_t)ny0 << L);
    grid_.assign((size_t)off_[ndense_], -1);
  }
  int get(int L, int i, int j) const {
    if (L < 0 || L >= nlev_ || i < 0 || j < 0 || i >= (nx0_ << L) || j >= (ny0_ << L)) return -1;
    if (L < ndense_) return grid_[(size_t)(off_[L] + (int64_t)j * (nx0_ << L) + i)];
    auto it = map_.find(key(L, i, j));
    return it == map_.end() ? -1 : it->second;
  }
  void set(int L, int i, int j, int v) {
    if (L < ndense_) grid_[(size_t)(off_[L] + (int64_t)j * (nx0_ << L) + i)] = v;
    else map_[key(L, i, j)] = v;
  }

 private:
  int nx0_, ny0_, nlev_, ndense_ = 0;
  std::vector<int64_t> off_;
  std::vector<int> grid_;
  std::unordered_map<int64_t, int> map_;
};


// Split [0, n) into chunks of at most `cap` items that do not cross a change of
// member; chunks are listed member by member.  Output: chunk (begin, length)
// pairs and the first chunk of every member (m0[M] = number of chunks).
void make_chunks(const std::vector<int>& mem_of, int M, int cap, std::vector<int>& ch, std::vector<int>& m0) {
  std::vector<std::vector<int>> per(M);
  const int n = (int)mem_of.size();
  int i = 0;
  while (i < n) {
    const int m = mem_of[i];
    int j = i + 1;
    while (j < n && j - i < cap && mem_of[j] == m) ++j;
    per[m].push_back(i);
    per[m].push_back(j - i);
    i = j;
  }
  ch.clear();
  m0.assign(M + 1, 0);
  for (int m = 0; m < M; ++m) {
    m0[m] = (int)ch.size() / 2;
    ch.insert(ch.end(), per[m].begin(), per[m].end());
  }
  m0[M] = (int)ch.size() / 2;
}

// Device tables depend only on (device, r, rule, S, volume rule): they are
// built once per process and shared by every context (a remesh then builds
// none); the cache owns them until the process ends.
struct TabEntry {
  std::vector<double> xh, wh, xv, wv;
  double w1;
  LevelTabs tabs, vtabs;
  double *d_tab, *d_vtab, *d_xh, *d_xv;
};
std::mutex g_tab_mu;
std::unordered_map<int64_t, TabEntry> g_tabs;

template <class T>
hipError_t tab_alloc(T** p, size_t n) {
  return hipMalloc((void**)p, std::max(n, (size_t)1) * sizeof(T));
}

sw_status build_tables_uncached(sw_ctx* c, LevelH& L);

sw_status build_tables(sw_ctx* c, LevelH& L) {
  const int64_t k = ((int64_t)c->dev << 40) | ((int64_t)c->r << 32) | ((int64_t)c->p.rule << 24) |
                    ((int64_t)L.S << 8) | (int64_t)c->nv;
  std::lock_guard<std::mutex> g(g_tab_mu);
  auto it = g_tabs.find(k);
  if (it == g_tabs.end()) {
    sw_status st = build_tables_uncached(c, L);
    if (st != SW_OK) return st;
    g_tabs[k] = TabEntry{L.xh, L.wh, L.xv, L.wv, L.w1, L.tabs, L.vtabs, L.d_tab, L.d_vtab, L.d_xh, L.d_xv};
    return SW_OK;
  }
  const TabEntry& e = it->second;
  L.xh = e.xh;
  L.wh = e.wh;
  L.xv = e.xv;
  L.wv = e.wv;
  L.w1 = e.w1;
  L.tabs = e.tabs;
  L.vtabs = e.vtabs;
  L.d_tab = e.d_tab;
  L.d_vtab = e.d_vtab;
  L.d_xh = e.d_xh;
  L.d_xv = e.d_xv;
  return SW_OK;
}

sw_status build_tables_uncached(sw_ctx* c, LevelH& L) {
  const int S = L.S, N1 = c->N1, NP = c->NP;
  if (c->p.rule == SW_RULE_EQ) eqr(S, L.xh, L.wh);
  else gll(S, L.xh, L.wh);
  std::vector<double> wb, xi;
  gll(N1, xi, wb);          // support points
  std::vector<double> tab;
  const size_t o_w = 0, o_l = o_w + S, o_d = o_l + (size_t)S * N1, o_m0 = o_d + (size_t)S * N1,
               o_mq = o_m0 + (size_t)NP * NP, o_mean = o_mq + (size_t)NP * NP, o_fl = o_mean + NP,
               o_wl = o_fl + (size_t)3 * S * N1, o_wd = o_wl + (size_t)S * N1, o_mqf = o_wd + (size_t)S * N1,
               total = o_mqf + (size_t)NP * NP;
  tab.assign(total, 0.0);
  for (int a = 0; a < S; ++a) {
    tab[o_w + a] = L.wh[a];
    for (int k = 0; k < N1; ++k) {
      tab[o_l + a * N1 + k] = lag(xi, k, L.xh[a]);
      tab[o_d + a * N1 + k] = dlag(xi, k, L.xh[a]);
      tab[o_fl + (0 * S + a) * N1 + k] = lag(xi, k, L.xh[a]);
      tab[o_fl + (1 * S + a) * N1 + k] = lag(xi, k, 0.5 * L.xh[a]);
      tab[o_fl + (2 * S + a) * N1 + k] = lag(xi, k, 0.5 * (1.0 + L.xh[a]));
      tab[o_wl + a * N1 + k] = L.wh[a] * lag(xi, k, L.xh[a]);
      tab[o_wd + a * N1 + k] = L.wh[a] * dlag(xi, k, L.xh[a]);
    }
  }
  // all-wet mass matrix of the sample rule on the unit square, and its inverse
  std::vector<double> M0(NP * NP, 0.0), Mq(NP * NP, 0.0);
  for (int i = 0; i < NP; ++i)
    for (int j = 0; j < NP; ++j) {
      double s = 0.0;
      for (int b = 0; b < S; ++b)
        for (int a = 0; a < S; ++a)
          s += L.wh[a] * L.wh[b] * tab[o_l + a * N1 + i % N1] * tab[o_l + b * N1 + i / N1] *
               tab[o_l + a * N1 + j % N1] * tab[o_l + b * N1 + j / N1];
      M0[i * NP + j] = s;
    }
  // exact mass matrix (Gauss-Legendre with r+1 points per direction, Table 1)
  std::vector<double> xg, wg;
  gl(N1, xg, wg);
  std::vector<double> mean(NP, 0.0);
  for (int i = 0; i < NP; ++i)
    for (int j = 0; j < NP; ++j) {
      double s = 0.0;
      for (int b = 0; b < N1; ++b)
        for (int a = 0; a < N1; ++a)
          s += wg[a] * wg[b] * lag(xi, i % N1, xg[a]) * lag(xi, i / N1, xg[b]) * lag(xi, j % N1, xg[a]) *
               lag(xi, j / N1, xg[b]);
      Mq[i * NP + j] = s;
    }
  for (int j = 0; j < NP; ++j) {
    double s = 0.0;
    for (int b = 0; b < N1; ++b)
      for (int a = 0; a < N1; ++a) s += wg[a] * wg[b] * lag(xi, j % N1, xg[a]) * lag(xi, j / N1, xg[b]);
    mean[j] = s;
  }
  for (int i = 0; i < NP * NP; ++i) tab[o_mqf + i] = Mq[i];
  if (!spd_inverse(M0, NP) || !spd_inverse(Mq, NP)) return fail(SW_EINVAL, "reference mass matrix not SPD");
  for (int i = 0; i < NP * NP; ++i) {
    tab[o_m0 + i] = M0[i];
    tab[o_mq + i] = Mq[i];
  }
  for (int j = 0; j < NP; ++j) tab[o_mean + j] = mean[j];
  sw_status st = SW_OK;
  HIPCHK(tab_alloc(&L.d_tab, total));
  HIPCHK(hipMemcpy(L.d_tab, tab.data(), total * sizeof(double), hipMemcpyHostToDevice));
  L.tabs.w = L.d_tab + o_w;
  L.tabs.l = L.d_tab + o_l;
  L.tabs.d = L.d_tab + o_d;
  L.tabs.m0inv = L.d_tab + o_m0;
  L.tabs.mqinv = L.d_tab + o_mq;
  L.tabs.meanw = L.d_tab + o_mean;
  L.tabs.fl = L.d_tab + o_fl;
  L.tabs.wl = L.d_tab + o_wl;
  L.tabs.wd = L.d_tab + o_wd;
  L.tabs.mq = L.d_tab + o_mqf;
  L.tabs.S = S;
  L.w1 = L.wh[0];
  L.vtabs = L.tabs;
  HIPCHK(tab_alloc(&L.d_xh, (size_t)S));
  HIPCHK(hipMemcpy(L.d_xh, L.xh.data(), S * sizeof(double), hipMemcpyHostToDevice));
  if (c->nv > 0) {
    // the volume terms' Gauss-Legendre rule (Table 1): weights, basis values
    // and derivatives at its nodes, and their weighted forms; the mass-matrix
    // entries stay the sample rule's (unused with this rule)
    const int nv = c->nv;
    gl(nv, L.xv, L.wv);
    const size_t v_w = 0, v_l = nv, v_d = v_l + (size_t)nv * N1, v_wl = v_d + (size_t)nv * N1,
                 v_wd = v_wl + (size_t)nv * N1, vtotal = v_wd + (size_t)nv * N1;
    std::vector<double> vt(vtotal, 0.0);
    for (int a = 0; a < nv; ++a) {
      vt[v_w + a] = L.wv[a];
      for (int k = 0; k < N1; ++k) {
        vt[v_l + a * N1 + k] = lag(xi, k, L.xv[a]);
        vt[v_d + a * N1 + k] = dlag(xi, k, L.xv[a]);
        vt[v_wl + a * N1 + k] = L.wv[a] * lag(xi, k, L.xv[a]);
        vt[v_wd + a * N1 + k] = L.wv[a] * dlag(xi, k, L.xv[a]);
      }
    }
    HIPCHK(tab_alloc(&L.d_vtab, vtotal));
    HIPCHK(hipMemcpy(L.d_vtab, vt.data(), vtotal * sizeof(double), hipMemcpyHostToDevice));
    L.vtabs.w = L.d_vtab + v_w;
    L.vtabs.l = L.d_vtab + v_l;
    L.vtabs.d = L.d_vtab + v_d;
    L.vtabs.wl = L.d_vtab + v_wl;
    L.vtabs.wd = L.d_vtab + v_wd;
    L.vtabs.fl = nullptr;
    L.vtabs.S = nv;
    HIPCHK(tab_alloc(&L.d_xv, (size_t)nv));
    HIPCHK(hipMemcpy(L.d_xv, L.xv.data(), nv * sizeof(double), hipMemcpyHostToDevice));
  }
  return SW_OK;
}

sw_status check_ptr(const void* p, const char* name) {
  if (!p) return fail(SW_EINVAL, std::string(name) + " is NULL");
  return SW_OK;
}

StageArgs stage_args(sw_ctx* c, const LevelH& L) {
  StageArgs a{};
  a.t = L.tabs;
  a.cell0 = L.cell0;
  a.ncell = L.ncell;
  a.K = c->K;
  a.zb = c->d_zb + L.off;
  a.vol = c->nv > 0 ? 1 : 0;
  a.tv = L.vtabs;
  a.zbv = c->d_zb + L.voff;
  a.bvec = c->d_bvec;
  a.zmax = c->d_zmax;
  a.nman = c->d_nman;
  a.cdx = c->d_cdx;
  a.cmem = c->d_cmem;
  a.mdt = c->d_mdt;
  for (int f = 0; f < 4; ++f) {
    a.sn[f] = c->d_sn[f];
    a.ss[f] = c->d_ss[f];
    a.in[f] = nullptr;
    a.out[f] = nullptr;
  }
  a.hn = c->d_hn;
  a.cn = c->d_cn;
  a.res = c->d_res;
  a.flag = c->d_flag;
  a.oflag = c->d_oflag;
  a.need = nullptr;
  a.wflag = nullptr;
  a.nwave = 0;
  for (int f = 0; f < 3; ++f) {
    a.replay[f] = c->rp[f];
    a.rec_end[f] = c->rec[f];
  }
  a.cdiag = c->d_cdiag;
  a.diag_init = 0;
  a.allwet = c->d_allwet;
  a.err = c->d_err;
  a.slot = 0;
  a.nterm = 0;
  a.g = c->p.g;
  a.eps = c->p.eps;
  a.hlim = c->p.h_lim;
  a.eps0 = c->p.eps0;
  a.newton_max = c->p.newton_max;
  a.tracer = c->p.tracer ? 1 : 0;
  a.tnu = c->p.tracer ? c->p.tracer_diff * c->p.tracer_strain / (double)(c->r * c->r) : 0.0;
  a.tkap = c->p.tracer ? c->p.tracer_decay : 0.0;
  a.fric = 1;
  a.adapt = c->p.adapt_degree ? 1 : 0;
  // contiguous cell ranges per XCD on single-level meshes; on quadtrees the
  // cost per cell clusters by region (dry land, refinement), and the
  // round-robin order balances it better across the XCDs (unless set)
  a.xmap = L.xorder >= 0 ? L.xorder : (c->lv.size() == 1 ? 1 : 0);
  a.imex = c->imex ? 1 : 0;
  a.lres = c->d_lres;
  a.gam = c->d_gam;
  for (int m = 0; m < 4; ++m) a.at[m] = 0.0;
  a.att = 0.0;
  return a;
}

// Face launch of one conflict-free group over the levels whose face kernel
// uses q lanes per face: direction dir (0: x faces, sides west/east; 1: y
// faces), second = 0: conforming and boundary faces with the first hanging
// sub-faces (classes 3 dir and 3 dir + 1, adjacent in the face order);
// second = 1: the second hanging sub-faces (class 3 dir + 2).  A cell side
// carries one face or two sub-faces, and sides of one direction touch disjoint
// dofs, so no two faces of a group touch the same (cell, dof).  nblk: the
// launch's workgroups (0: nothing to do).
FaceArgs face_args(sw_ctx* c, int dir, int second, int q, const double* const* st, double cstage, int slot,
                   int& nblk) {
  FaceArgs a{};
  a.K = c->K;
  const int fpb = kWave / q, k0 = 3 * dir + (second ? 2 : 0);
  int blk = 0, ns = 0;
  for (auto& L : c->lv) {
    if (L.face_q != q) continue;
    const int n = second ? L.cnface[k0] : L.cnface[k0] + L.cnface[k0 + 1];
    if (n == 0) continue;
    a.sblk[ns] = blk;
    a.sface0[ns] = L.cface0[k0];
    a.snface[ns] = n;
    a.sS[ns] = L.S;
    a.sfl[ns] = L.tabs.fl;
    a.sw[ns] = L.tabs.w;
    a.szf[ns] = c->d_zf + L.zfoff + (size_t)(L.cface0[k0] - L.face0) * 2 * L.S;
    blk += (n + fpb - 1) / fpb;
    ++ns;
  }
  a.sblk[ns] = blk;
  a.nseg = ns;
  nblk = blk;
  a.fA = c->d_fA;
  a.fB = c->d_fB;
  a.meta = c->d_meta;
  for (int f = 0; f < 4; ++f) a.st[f] = st[f];
  a.res = c->d_res;
  a.slot = slot;
  a.cdx = c->d_cdx;
  a.cw1 = c->d_cw1;
  a.cmem = c->d_cmem;
  a.mt = c->d_mt;
  a.mdt = c->d_mdt;
  a.mtide = c->d_mtide;
  a.cstage = cstage;
  a.fdt = c->d_fdt;
  a.err = c->d_err;
  a.g = c->p.g;
  a.eps = c->p.eps;
  a.tracer = c->p.tracer ? 1 : 0;
  a.tonly = (c->p.tracer && c->replaying) ? 1 : 0;
  a.gof = c->d_gof;
  a.ghost = c->d_ghost;
  a.ng = c->ng;
  a.xmap = 1;
  return a;
}

// all faces of all levels, adding into residual slot `slot`: x faces, then y
// faces, each as the conforming/first-sub-face group and the second-sub-face
// group (one launch per group and face-lane count)
sw_status faces(sw_ctx* c, const double* const* st, double cstage, int slot, const double* mt_override = nullptr) {
  std::vector<int> qs;
  for (auto& L : c->lv)
    if (std::find(qs.begin(), qs.end(), L.face_q) == qs.end()) qs.push_back(L.face_q);
  int n = 0;
  for (int dir = 0; dir < 2; ++dir)
    for (int second = 0; second < 2; ++second)
      for (int q : qs) {
        int nblk = 0;
        (void)face_args(c, dir, second, q, st, cstage, slot, nblk);
        n += nblk > 0;
      }
  sw_ctx::Scope sc(c, 3, n);
  for (int dir = 0; dir < 2; ++dir)
    for (int second = 0; second < 2; ++second)
      for (int q : qs) {
        int nblk = 0;
        FaceArgs fa = face_args(c, dir, second, q, st, cstage, slot, nblk);
        if (nblk == 0) continue;
        if (mt_override) fa.mt = mt_override;
        HIPCHK(launch_face(c->r, q, fa, nblk, c->s));
      }
  return SW_OK;
}

// per-member dt = cfl_m * min of the member's face bounds (two-level segmented
// reduction; mcfl == nullptr gives the bare bound)
sw_status reduce_dt(sw_ctx* c, const double* mcfl, double* dst) {
  if (c->nfch > 0) {
    hipLaunchKernelGGL(k_minred_seg, dim3(c->nfch), dim3(256), 0, c->s, c->d_fdt, c->d_fch, c->d_part);
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_dt_seg, dim3(c->M), dim3(256), 0, c->s, c->d_part, c->d_fch_m0, mcfl, dst);
  HIPCHK(hipGetLastError());
  return SW_OK;
}

// element work of one phase on every level: the fast kernel where it applies,
// then the general kernel on the cells it left (or on all cells)
// IMEX: coeft are the implicit weights of the combination and att its
// diagonal weight
sw_status elements(sw_ctx* c, int fmode, int gmode, int gmode2, int slot, int nterm, const double* coef, int diag_init,
                   int kind, const double* coeft = nullptr, double att = 0.0) {
  // a tracer replay, and the volume terms on a rule of their own, run the
  // general kernel on every cell; a replay's stages (no degree decision or
  // remap) run the fast tracer kernel on every cell, with the flow from the
  // record
  const bool tracer = c->p.tracer != 0;
  const bool replay = tracer && c->rp[0] != nullptr;
  const bool fast_ok = !replay && c->nv == 0;
  const bool trc_replay = replay && fmode == F_STAGE && c->nv == 0;
  // a replay's final combination: the degree decision on the recorded end
  // flow, the fast tracer kernel on the cells that keep their degree, the
  // general kernel (final combination and next start) on the others
  const bool trc_final = replay && fmode == F_FINAL && c->nv == 0;
  if ((fast_ok && tracer && fmode == F_FINAL) || trc_final) {
    // the final kernel updates the degree flags; the tracer kernel reads the step's own
    hipLaunchKernelGGL(k_copy8, dim3((c->K + 255) / 256), dim3(256), 0, c->s, c->d_flag, c->d_oflag, (size_t)c->K);
    HIPCHK(hipGetLastError());
  }
  for (auto& L : c->lv) {
    StageArgs a = stage_args(c, L);
    a.slot = slot;
    a.nterm = nterm;
    for (int m = 0; m < 4; ++m) a.a[m] = coef ? coef[m] : 0.0;
    for (int m = 0; m < 4; ++m) a.at[m] = coeft ? coeft[m] : 0.0;
    a.att = att;
    a.diag_init = diag_init;
    if (fast_ok) {
      sw_ctx::Scope sc(c, kind, 1);
      a.need = c->d_need;
      a.wflag = L.d_wflag;
      a.nwave = L.nblk;
      const int wpb = c->imex ? 1 : L.wpb;   // the IMEX variant runs one wavefront per workgroup
      const int cpb = wpb * kWave / L.P;
      HIPCHK(launch_elem(c->r, L.P, fmode, wpb, a, (L.ncell + cpb - 1) / cpb, c->s));
    }
    if (fast_ok && tracer) {
      // tracer solve, C~ and tracer residual of the cells the fast kernel kept
      sw_ctx::Scope sc(c, fmode == F_STAGE ? 5 : 6, 1);
      StageArgs tr = a;
      tr.need = c->d_need;
      HIPCHK(launch_trc(c->r, L.P, fmode, tr, L.nblk, c->s));
    }
    if (trc_replay) {
      sw_ctx::Scope sc(c, 5, 1);
      StageArgs tr = a;
      tr.need = nullptr;   // every cell
      HIPCHK(launch_trc(c->r, L.P, F_STAGE, tr, L.nblk, c->s));
      continue;
    }
    if (trc_final) {
      StageArgs d = a;
      d.need = c->d_need;
      d.wflag = L.d_wflag;
      HIPCHK(launch_trc_degree(c->r, L.P, d, L.nblk, c->s));
      {
        sw_ctx::Scope sc(c, 6, 1);
        StageArgs tr = a;
        tr.need = c->d_need;   // the cells that keep their degree
        HIPCHK(launch_trc(c->r, L.P, F_FINAL, tr, L.nblk, c->s));
      }
      sw_ctx::Scope sc(c, 4, 1);
      StageArgs g = a;
      g.need = c->d_need;
      g.wflag = L.d_wflag;
      g.nwave = L.nblk;
      HIPCHK(launch_stage_scan(c->r, L.P, gmode, gmode2, g, std::min(L.nblk, kListGrid), c->s));
      continue;
    }
    StageArgs g = a;
    g.need = fast_ok ? c->d_need : nullptr;
    g.wflag = nullptr;
    g.nwave = 0;
    if (fast_ok) {
      // the wavefronts the fast kernel flagged, walked by a small grid (both
      // modes in one launch)
      if (gmode >= 0) {
        sw_ctx::Scope sc(c, 4, 1);
        g.wflag = L.d_wflag;
        g.nwave = L.nblk;
        HIPCHK(launch_stage_scan(c->r, L.P, gmode, gmode2, g, std::min(L.nblk, kListGrid), c->s));
      }
    } else {
      if (gmode >= 0) {
        sw_ctx::Scope sc(c, 4, 1);
        HIPCHK(launch_stage(c->r, L.P, gmode, g, L.nblk, c->s));
      }
      if (gmode2 >= 0) {
        sw_ctx::Scope sc(c, 4, 1);
        g.slot = 0;
        HIPCHK(launch_stage(c->r, L.P, gmode2, g, L.nblk, c->s));
      }
    }
  }
  return SW_OK;
}

sw_status rebake(sw_ctx* c) {
  c->start_ready = false;
  for (auto& L : c->lv) {
    const size_t n = (size_t)L.ncell * L.S * L.S;
    if (n == 0) continue;
    hipLaunchKernelGGL(k_bathy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->s, c->d_braw, c->d_db, c->d_zb,
                       L.cell0, L.ncell, L.S, L.off);
    HIPCHK(hipGetLastError());
    if (c->nv > 0) {   // the volume rule's depth samples
      const size_t nvn = (size_t)L.ncell * c->nv * c->nv;
      hipLaunchKernelGGL(k_bathy, dim3((unsigned)((nvn + 255) / 256)), dim3(256), 0, c->s, c->d_braw, c->d_db,
                         c->d_zb, L.cell0, L.ncell, c->nv, L.voff);
      HIPCHK(hipGetLastError());
    }
  }
  for (auto& L : c->lv) {
    if (L.nface > 0) {
      const int n = L.nface * L.S;   // all classes of the level: one contiguous range
      hipLaunchKernelGGL(k_facez, dim3((n + 255) / 256), dim3(256), 0, c->s, c->d_fA, c->d_fB, c->d_meta, L.face0,
                         L.nface, L.S, L.cell0, L.ncell, L.off, c->d_zb, c->d_braw, c->d_db, c->d_zf + L.zfoff,
                         c->d_err, c->K);
      HIPCHK(hipGetLastError());
    }
    if (L.ncell > 0) {
      const int n = L.ncell * c->NP;
      hipLaunchKernelGGL(k_cellinit, dim3((n + 127) / 128), dim3(128), 0, c->s, L.tabs, L.cell0, L.ncell, L.off,
                         c->N1, c->d_zb, c->d_cdx, c->d_bvec, c->d_zmax);
      HIPCHK(hipGetLastError());
    }
  }
  return SW_OK;
}

sw_status need_bathy(const sw_ctx* c) {
  if (!c->bathy_set) return fail(SW_EINVAL, "sw_set_bathymetry has not been called");
  return SW_OK;
}

// bathymetry and, with state or discharge sides, their boundary data
sw_status need_inputs(const sw_ctx* c) {
  sw_status st = need_bathy(c);
  if (st != SW_OK) return st;
  if (c->ng > 0 && !c->ghost_set)
    return fail(SW_EINVAL, "the mesh has state or discharge sides: call sw_set_boundary_state first");
  return SW_OK;
}

}  // namespace

// Device scratch of sw_apply_operator_noalloc, one copy per GPU for the life
// of the process (48 MiB).  Host code never passes `scratch` itself to a
// kernel: its name is a host-side stand-in, and each device's address is
// fetched once (scratch_setup, from sw_create with that device current) and
// kept in g_scratch[device].
constexpr size_t kScratchDoubles = (size_t)6 << 20;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// the current device's copy of the scratch array (hipGetSymbolAddress, once)
sw_status scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(SW_EINVAL, "device index out of the library's range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[dev]) return SW_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return fail(SW_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch[dev] = static_cast<double*>(ptr);
  return SW_OK;
}

double* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[dev];
}
}  // namespace

extern "C" {

const char* sw_last_error(void) { return g_err.c_str(); }

// trusted: the meshes come from the library's own remesh plan (sorted,
// in range, tiling, 2:1 balanced by construction), so the per-cell
// duplicate, tiling and one-face-per-side checks are skipped
static sw_status create_ctx(sw_ctx** out, int32_t n_members, const sw_mesh_desc* meshes, const sw_params* params,
                            void* stream, bool trusted) {
  if (!out || !meshes || !params) return fail(SW_EINVAL, "NULL argument to sw_create_batch");
  *out = nullptr;
  if (n_members < 1) return fail(SW_EINVAL, "n_members must be >= 1");
  const sw_params* p = &params[0];
  if (p->r < 1 || p->r > 3) return fail(SW_EINVAL, "r must be 1, 2 or 3");
  if (p->rule != SW_RULE_EQ && p->rule != SW_RULE_GLL) return fail(SW_EINVAL, "unknown rule");
  if (p->rk < SW_RK_FE || p->rk > SW_RK_IMEX) return fail(SW_EINVAL, "unknown RK scheme");
  if (!(p->eps > 0.0)) return fail(SW_EINVAL, "eps must be > 0");
  if (p->newton_max < 1 || p->newton_max > 1000) return fail(SW_EINVAL, "newton_max out of range");
  if (p->n_levels < 1 || p->n_levels > 8) return fail(SW_EINVAL, "n_levels must be 1..8");
  if (!(p->tracer_diff >= 0.0 && p->tracer_diff < 1e300) || !(p->tracer_strain >= 0.0 && p->tracer_strain < 1e300) ||
      !(p->tracer_decay >= 0.0 && p->tracer_decay < 1e300))
    return fail(SW_EINVAL, "tracer_diff, tracer_strain and tracer_decay must be finite and >= 0");
  if (p->quadrature != SW_QUAD_SUBGRID && p->quadrature != SW_QUAD_PAPER)
    return fail(SW_EINVAL, "unknown quadrature");
  if (p->quadrature == SW_QUAD_PAPER) {
    // Table 1: faces and the continuity mass on GLL (r+2)^2
    if (p->rule != SW_RULE_GLL) return fail(SW_EINVAL, "the paper's quadrature takes the GLL rule (Table 1)");
    for (int L = 0; L < p->n_levels; ++L)
      if (p->S[L] != p->r + 2) return fail(SW_EINVAL, "the paper's quadrature takes S = r + 2 on every level");
  }
  for (int m = 0; m < n_members; ++m) {
    const sw_params& q = params[m];
    bool same = q.r == p->r && q.rule == p->rule && q.rk == p->rk && q.n_levels == p->n_levels && q.g == p->g &&
                q.eps == p->eps && q.h_lim == p->h_lim && q.eps0 == p->eps0 && q.newton_max == p->newton_max &&
                q.cfl_mode == p->cfl_mode && (q.tracer != 0) == (p->tracer != 0) &&
                (q.adapt_degree != 0) == (p->adapt_degree != 0) && q.tracer_diff == p->tracer_diff &&
                q.tracer_strain == p->tracer_strain && q.tracer_decay == p->tracer_decay &&
                q.quadrature == p->quadrature;
    for (int L = 0; L < p->n_levels; ++L) same = same && q.S[L] == p->S[L];
    if (!same)
      return fail(SW_EINVAL, "member " + std::to_string(m) +
                                 ": members of one batch must share r, rule, rk, S, g, eps, h_lim, eps0, newton_max, "
                                 "cfl_mode, tracer, adapt_degree, the tracer diffusion and decay and the "
                                 "quadrature");
    const sw_mesh_desc& md = meshes[m];
    const bool elev = md.bc[0] == SW_BC_ELEV || md.bc[1] == SW_BC_ELEV || md.bc[2] == SW_BC_ELEV ||
                      md.bc[3] == SW_BC_ELEV;
    if (q.tide_period == 0.0 && elev)
      return fail(SW_EINVAL, "tide_period must be non-zero with an elevation boundary");
    if (md.n_cells < 1 || !md.level || !md.i || !md.j) return fail(SW_EINVAL, "empty mesh");
    if (md.nx0 < 1 || md.ny0 < 1 || !(md.dx0 > 0.0)) return fail(SW_EINVAL, "bad coarse grid");
    for (int sd = 0; sd < 4; ++sd)
      if (md.bc[sd] < 0 || md.bc[sd] > SW_BC_DISCHARGE) return fail(SW_EINVAL, "bad boundary kind");
    if ((md.bc[0] == SW_BC_PERIODIC) != (md.bc[1] == SW_BC_PERIODIC) ||
        (md.bc[2] == SW_BC_PERIODIC) != (md.bc[3] == SW_BC_PERIODIC))
      return fail(SW_EINVAL, "periodic boundaries must come in pairs");
  }
  auto* c = new sw_ctx();
  auto bail = [&](sw_status st, const std::string& msg) {
    delete c;
    return fail(st, msg);
  };
  c->s = (hipStream_t)stream;
  {
    hipError_t e = hipGetDevice(&c->dev);
    if (e != hipSuccess) return bail(SW_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    // the device scratch of sw_apply_operator_noalloc on this device
    if (scratch_setup(c->dev) != SW_OK) {
      delete c;
      return SW_EHIP;
    }
  }
  c->p = *p;
  c->M = n_members;
  c->r = p->r;
  c->N1 = p->r + 1;
  c->NP = c->N1 * c->N1;
  tableau(p->rk, c->ns, c->A, c->b, c->c);
  implicit_tableau(p->rk, c->At);
  c->imex = p->rk == SW_RK_IMEX;
  const int M = n_members;
  // per-member validation: level order, extent, tiling, duplicates
  int maxL = 0;
  int64_t Ktot = 0;
  std::vector<LeafIndex> leaf;
  leaf.reserve(M);
  for (int m = 0; m < M; ++m) {
    const sw_mesh_desc& md = meshes[m];
    c->mx0.push_back(md.x0);
    c->my0.push_back(md.y0);
    c->mdx0.push_back(md.dx0);
    c->mnx0.push_back(md.nx0);
    c->mny0.push_back(md.ny0);
    c->mbc.push_back({md.bc[0], md.bc[1], md.bc[2], md.bc[3]});
    // area in units of the finest level's cells (exact in integers)
    const int sh = 2 * (p->n_levels - 1);
    int64_t area = 0;
    if (md.nx0 < 1 || md.ny0 < 1) return bail(SW_EINVAL, "bad coarse grid");
    leaf.emplace_back(md.nx0, md.ny0, p->n_levels, p->n_levels);
    for (int k = 0; k < md.n_cells; ++k) {
      const int L = md.level[k];
      if (L < 0 || L >= p->n_levels) return bail(SW_EINVAL, "cell level out of range (n_levels)");
      if (k > 0 && L < md.level[k - 1]) return bail(SW_EINVAL, "cells must be sorted by level");
      if (md.i[k] < 0 || md.j[k] < 0 || md.i[k] >= (md.nx0 << L) || md.j[k] >= (md.ny0 << L))
        return bail(SW_EINVAL, "cell outside the domain");
      maxL = std::max(maxL, L);
      area += (int64_t)1 << (sh - 2 * L);
      if (!trusted && leaf[m].get(L, md.i[k], md.j[k]) != -1) return bail(SW_EINVAL, "duplicate cell");
      leaf[m].set(L, md.i[k], md.j[k], k);
    }
    if (!trusted && area != ((int64_t)md.nx0 * md.ny0) << sh)
      return bail(SW_EINVAL, "cells do not tile the domain");
    Ktot += md.n_cells;
  }
  if (Ktot > (int64_t)1 << 30) return bail(SW_EINVAL, "too many cells");
  c->K = (int)Ktot;
  const int K = c->K;
  // levels (sample counts shared by the members)
  for (int L = 0; L <= maxL; ++L) {
    LevelH h;
    h.L = L;
    h.S = p->S[L];
    if (h.S < p->r + 2 || h.S > 32) return bail(SW_EINVAL, "S must satisfy r+2 <= S <= 32 on every level");
    h.P = lanes_for(h.S);
    c->lv.push_back(h);
  }
  // context order: level, then member, then the member's own order
  std::vector<std::vector<int>> ctx_of(M);
  for (int m = 0; m < M; ++m) ctx_of[m].assign(meshes[m].n_cells, -1);
  {
    int64_t off = 0;
    c->cmem.reserve(K);
    c->cloc.reserve(K);
    c->lev.reserve(K);
    c->ci.reserve(K);
    c->cj.reserve(K);
    c->cdx.reserve(K);
    // each member's cells are sorted by level: one cursor per member
    std::vector<int> cur(M, 0);
    for (auto& L : c->lv) {
      L.cell0 = (int)c->cmem.size();
      for (int m = 0; m < M; ++m) {
        const sw_mesh_desc& md = meshes[m];
        const double dxl = md.dx0 / std::ldexp(1.0, L.L);
        int k = cur[m];
        for (; k < md.n_cells && md.level[k] == L.L; ++k) {
          ctx_of[m][k] = (int)c->cmem.size();
          c->cmem.push_back(m);
          c->cloc.push_back(k);
          c->lev.push_back(L.L);
          c->ci.push_back(md.i[k]);
          c->cj.push_back(md.j[k]);
          c->cdx.push_back(dxl);
        }
        cur[m] = k;
      }
      L.ncell = (int)c->cmem.size() - L.cell0;
      L.off = (size_t)off;
      off += (int64_t)L.ncell * L.S * L.S;
    }
    c->nvol = off;
    // the volume rule of Table 1 has floor(3r/2)+1 Gauss-Legendre points per
    // direction; its samples follow the sample nodes, cell by cell
    c->nv = p->quadrature == SW_QUAD_PAPER ? (3 * p->r) / 2 + 1 : 0;
    for (auto& L : c->lv) L.voff = (size_t)c->nvol + (size_t)L.cell0 * c->nv * c->nv;
    c->nvv = (int64_t)K * c->nv * c->nv;
  }
  // faces: conforming (recorded from the W/S cell), hanging (from the fine cell),
  // boundary; A is the fine or equal side.  Faces join cells of one member only.
  struct FaceH { int a, b, sa, sb, sub, bnd, bc, lvl; };
  std::vector<FaceH> fh;
  fh.reserve((size_t)K * 3);
  const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1}, opp[4] = {1, 0, 3, 2};
  for (int k = 0; k < K; ++k) {
    const int m = c->cmem[k];
    const sw_mesh_desc& md = meshes[m];
    const bool perx = md.bc[0] == SW_BC_PERIODIC, pery = md.bc[2] == SW_BC_PERIODIC;
    const int L = c->lev[k], i = c->ci[k], j = c->cj[k];
    const int nxL = md.nx0 << L, nyL = md.ny0 << L;
    for (int sd = 0; sd < 4; ++sd) {
      int ni = i + di[sd], nj = j + dj[sd];
      bool outside = false;
      if (ni < 0 || ni >= nxL) {
        if (perx) ni = (ni + nxL) % nxL;
        else outside = true;
      }
      if (nj < 0 || nj >= nyL) {
        if (pery) nj = (nj + nyL) % nyL;
        else outside = true;
      }
      if (outside) {
        fh.push_back({k, -1, sd, 0, -1, 1, md.bc[sd], L});
        continue;
      }
      const int it = leaf[m].get(L, ni, nj);
      if (it >= 0) {
        if (sd == 1 || sd == 3) fh.push_back({k, ctx_of[m][it], sd, opp[sd], -1, 0, 0, L});
        continue;
      }
      if (L > 0) {
        const int ic = leaf[m].get(L - 1, ni >> 1, nj >> 1);
        if (ic >= 0) {
          const int sub = (sd < 2) ? (j & 1) : (i & 1);
          fh.push_back({k, ctx_of[m][ic], sd, opp[sd], sub, 0, 0, L});
          continue;
        }
      }
      // finer neighbour: both children along this side must be leaves
      bool ok = true;
      for (int t = 0; t < 2; ++t) {
        int ki, kj;
        if (sd < 2) {
          ki = 2 * ni + (sd == 0 ? 1 : 0);
          kj = 2 * nj + t;
        } else {
          ki = 2 * ni + t;
          kj = 2 * nj + (sd == 2 ? 1 : 0);
        }
        if (leaf[m].get(L + 1, ki, kj) < 0) ok = false;
      }
      if (!ok)
        return bail(SW_EINVAL, "mesh is not 2:1 balanced at cell " + std::to_string(c->cloc[k]) + " of member " +
                                   std::to_string(m));
    }
  }
  // class of a face: x or y direction times (conforming/boundary, sub-face 0, sub-face 1);
  // the stable sort keeps the faces of a class grouped by member
  auto cls = [](const FaceH& h) { return (h.sa < 2 ? 0 : 3) + (h.sub + 1); };
  {   // counting sort by (level, class), stable
    const int nb = 6 * (int)c->lv.size();
    std::vector<int> cnt(nb + 1, 0);
    for (const FaceH& h : fh) ++cnt[6 * h.lvl + cls(h) + 1];
    for (int b = 0; b < nb; ++b) cnt[b + 1] += cnt[b];
    std::vector<FaceH> sorted(fh.size());
    for (const FaceH& h : fh) sorted[cnt[6 * h.lvl + cls(h)]++] = h;
    fh.swap(sorted);
  }
  c->F = (int)fh.size();
  std::vector<int> fA(c->F), fB(c->F), meta(c->F), used(trusted ? 0 : (size_t)K * 8, 0), fmem(c->F);
  for (int f = 0; f < c->F; ++f) {
    const FaceH& h = fh[f];
    fA[f] = h.a;
    fB[f] = h.b;
    fmem[f] = c->cmem[h.a];
    meta[f] = h.sa | (h.sb << 2) | ((h.sub + 1) << 4) | (h.bnd << 6) | (h.bc << 8);
    if (h.bnd && (h.bc == SW_BC_STATE || h.bc == SW_BC_DISCHARGE)) {
      c->gface.push_back(f);
      c->gcell.push_back(h.a);
      c->gside.push_back(h.sa);
    }
    // every cell side carries one face, or two sub-faces on a coarse side
    if (trusted) continue;
    if (used[(size_t)h.a * 8 + h.sa * 2]++) return bail(SW_EINVAL, "two faces on one cell side");
    if (!h.bnd && used[(size_t)h.b * 8 + h.sb * 2 + (h.sub < 0 ? 0 : h.sub)]++)
      return bail(SW_EINVAL, "two faces on one cell side");
  }
  // chunks of the segmented reductions (faces: dt bounds; cells: diagnostics)
  std::vector<int> fch, fch_m0, cch, cch_m0;
  {
    make_chunks(fmem, M, kFaceChunk, fch, fch_m0);
    make_chunks(c->cmem, M, kCellChunk, cch, cch_m0);
    c->nfch = (int)fch.size() / 2;
    c->ncch = (int)cch.size() / 2;
  }
  size_t zo = 0;
  {
    int f = 0;
    for (auto& L : c->lv) {
      L.face0 = f;
      const int cpb = kWave / L.P;
      for (int k = 0; k < 6; ++k) {
        L.cface0[k] = f;
        while (f < c->F && fh[f].lvl == L.L && cls(fh[f]) == k) ++f;
        L.cnface[k] = f - L.cface0[k];
        L.cfnblk[k] = (L.cnface[k] + kWave / kFaceLanes - 1) / (kWave / kFaceLanes);
      }
      L.nface = f - L.face0;
      L.zfoff = zo;
      zo += (size_t)L.nface * 2 * L.S;
      L.nblk = (L.ncell + cpb - 1) / cpb;
    }
    if (f != c->F) return bail(SW_EINVAL, "internal: face classes do not cover the face list");
  }
  {
    sw_status st = SW_OK;
    const size_t KN = (size_t)K * c->NP;
#define ALLOC(ptr, n)                          \
  if ((st = c->alloc(&ptr, n)) != SW_OK) {     \
    delete c;                                  \
    return st;                                 \
  }
    ALLOC(c->d_fA, c->F);
    ALLOC(c->d_fB, c->F);
    ALLOC(c->d_meta, c->F);
    ALLOC(c->d_err, 1);
    ALLOC(c->d_cmem, K);
    ALLOC(c->d_ci, K);
    ALLOC(c->d_cj, K);
    ALLOC(c->d_mxy, (size_t)2 * M);
    ALLOC(c->d_zb, (size_t)(c->nvol + c->nvv));
    ALLOC(c->d_braw, (size_t)(c->nvol + c->nvv));
    ALLOC(c->d_db, K);
    ALLOC(c->d_bvec, KN);
    ALLOC(c->d_zmax, K);
    ALLOC(c->d_nman, K);
    ALLOC(c->d_cdx, K);
    ALLOC(c->d_cw1, K);
    ALLOC(c->d_zf, zo);
    for (int q = 0; q < 4; ++q) {
      ALLOC(c->d_sn[q], KN);
      ALLOC(c->d_ss[q], KN);
    }
    ALLOC(c->d_hn, KN);
    ALLOC(c->d_cn, KN);
    ALLOC(c->d_res, (size_t)kNSlot * 4 * KN);
    ALLOC(c->d_cdiag, (size_t)K * D_NSLOT);
    ALLOC(c->d_mt, M);
    ALLOC(c->d_mdt, M);
    ALLOC(c->d_mt_apply, M);
    ALLOC(c->d_mtide, (size_t)4 * M);
    ALLOC(c->d_mcfl, M);
    ALLOC(c->d_mdiag, (size_t)kMDiag * M);
    ALLOC(c->d_mtmp, M);
    ALLOC(c->d_fdt, c->F);
    ALLOC(c->d_part, (size_t)std::max(c->nfch, c->ncch) * D_NSLOT);
    ALLOC(c->d_fch, fch.size());
    ALLOC(c->d_fch_m0, M + 1);
    ALLOC(c->d_cch, cch.size());
    ALLOC(c->d_cch_m0, M + 1);
    ALLOC(c->d_need, K);
    ALLOC(c->d_flag, K);
    ALLOC(c->d_oflag, K);
    ALLOC(c->d_allwet, K);
    ALLOC(c->d_fdb, (size_t)2 * c->F);
    ALLOC(c->d_cfoff, (size_t)K + 1);
    ALLOC(c->d_cfent, (size_t)2 * c->F);
    ALLOC(c->d_gof, c->F);
    if (c->imex) {
      ALLOC(c->d_lres, (size_t)kNSlot * 2 * KN);
      ALLOC(c->d_gam, (size_t)K * (c->NP * (c->NP + 1) / 2));
    }
#undef ALLOC
  }
  for (auto& L : c->lv) {
    sw_status st = build_tables(c, L);
    if (st == SW_OK) st = c->alloc(&L.d_wflag, (size_t)std::max(L.nblk, 1));
    if (st != SW_OK) {
      delete c;
      return st;
    }
    hipError_t e = hipMemsetAsync(L.d_wflag, 0, (size_t)std::max(L.nblk, 1), c->s);
    if (e != hipSuccess) return bail(SW_EHIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
  }
  std::vector<double> cw1(K), mtide(4 * (size_t)M), mcfl(M);
  for (int k = 0; k < K; ++k) cw1[k] = p->cfl_mode == 1 ? c->lv[c->lev[k]].w1 : 1.0;
  for (int m = 0; m < M; ++m) {
    mtide[4 * m + 0] = params[m].tide_amp;
    mtide[4 * m + 1] = params[m].tide_period;
    mtide[4 * m + 2] = params[m].tide_phase;
    mtide[4 * m + 3] = params[m].tide_c_in;
    mcfl[m] = params[m].cfl;
  }
  // host data goes to the device through one pinned staging buffer with
  // asynchronous copies on the context's stream, awaited at the end
  Uploads up;
  up.blob.reserve(((size_t)40 * K + (size_t)28 * c->F + 4096) * 2);
#define H2D(dst, src, n) up.add((void*)(dst), (const void*)(src), (size_t)(n) * sizeof(*(src)))
#define ZERO(dst, bytes)                                                                       \
  do {                                                                                         \
    hipError_t e_ = hipMemsetAsync(dst, 0, bytes, c->s);                                       \
    if (e_ != hipSuccess) return bail(SW_EHIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e_)); \
  } while (0)
  {
    // node offsets of the faces with given boundary data (S nodes of the face's level)
    std::vector<int> gof(c->F, -1);
    int64_t o = 0;
    for (int f : c->gface) {
      gof[f] = (int)o;
      o += c->lv[c->lev[fA[f]]].S;
    }
    if (o > INT32_MAX / 4) return bail(SW_EINVAL, "too many boundary data nodes");
    c->ng = o;
    H2D(c->d_gof, gof.data(), c->F);
    if (c->ng > 0) {
      sw_status st = c->alloc(&c->d_ghost, (size_t)4 * c->ng);
      if (st != SW_OK) {
        delete c;
        return st;
      }
      ZERO(c->d_ghost, (size_t)4 * c->ng * sizeof(double));
    }
  }
  H2D(c->d_fA, fA.data(), c->F);
  H2D(c->d_fB, fB.data(), c->F);
  H2D(c->d_meta, meta.data(), c->F);
  H2D(c->d_cmem, c->cmem.data(), K);
  H2D(c->d_ci, c->ci.data(), K);
  H2D(c->d_cj, c->cj.data(), K);
  {
    std::vector<double> mxy(c->mx0);
    mxy.insert(mxy.end(), c->my0.begin(), c->my0.end());
    H2D(c->d_mxy, mxy.data(), (size_t)2 * M);
  }
  H2D(c->d_cdx, c->cdx.data(), K);
  H2D(c->d_cw1, cw1.data(), K);
  H2D(c->d_mtide, mtide.data(), 4 * (size_t)M);
  H2D(c->d_mcfl, mcfl.data(), M);
  H2D(c->d_fch, fch.data(), fch.size());
  H2D(c->d_fch_m0, fch_m0.data(), M + 1);
  H2D(c->d_cch, cch.data(), cch.size());
  H2D(c->d_cch_m0, cch_m0.data(), M + 1);
  {
    // cell -> entries of the per-face adjoint array: A side 2f, B side 2f+1
    std::vector<int> cnt((size_t)K + 1, 0), ent((size_t)2 * c->F);
    for (int f = 0; f < c->F; ++f) {
      ++cnt[fA[f] + 1];
      if (!fh[f].bnd) ++cnt[fB[f] + 1];
    }
    for (int k = 0; k < K; ++k) cnt[k + 1] += cnt[k];
    std::vector<int> pos(cnt.begin(), cnt.end() - 1);
    for (int f = 0; f < c->F; ++f) {
      ent[pos[fA[f]]++] = 2 * f;
      if (!fh[f].bnd) ent[pos[fB[f]]++] = 2 * f + 1;
    }
    H2D(c->d_cfoff, cnt.data(), (size_t)K + 1);
    if (cnt[K] > 0) H2D(c->d_cfent, ent.data(), (size_t)cnt[K]);
  }
  ZERO(c->d_err, sizeof(int));
  ZERO(c->d_db, sizeof(double) * K);
  ZERO(c->d_nman, sizeof(double) * K);
  ZERO(c->d_mt, sizeof(double) * M);
  ZERO(c->d_mdt, sizeof(double) * M);
  ZERO(c->d_mt_apply, sizeof(double) * M);
  ZERO(c->d_mdiag, sizeof(double) * kMDiag * M);
  ZERO(c->d_cdiag, sizeof(double) * (size_t)K * D_NSLOT);
  ZERO(c->d_need, K);
  ZERO(c->d_res, sizeof(double) * (size_t)kNSlot * 4 * K * c->NP);
  ZERO(c->d_allwet, K);
  for (int q = 0; q < 4; ++q) {
    ZERO(c->d_sn[q], sizeof(double) * K * c->NP);
    ZERO(c->d_ss[q], sizeof(double) * K * c->NP);
  }
  ZERO(c->d_hn, sizeof(double) * K * c->NP);
  ZERO(c->d_cn, sizeof(double) * K * c->NP);
  {
    hipError_t e = hipMemsetAsync(c->d_flag, c->r, K, c->s);
    if (e == hipSuccess) e = up.flush(c->dev, c->s);
    if (e == hipSuccess) e = hipStreamSynchronize(c->s);
    if (e != hipSuccess) return bail(SW_EHIP, std::string("context set-up: ") + hipGetErrorString(e));
  }
#undef H2D
#undef ZERO
  *out = c;
  return SW_OK;
}

sw_status sw_create_batch(sw_ctx** out, int32_t n_members, const sw_mesh_desc* meshes, const sw_params* params,
                          void* stream) {
  return create_ctx(out, n_members, meshes, params, stream, false);
}

sw_status sw_create(sw_ctx** out, const sw_mesh_desc* m, const sw_params* p, void* stream) {
  return sw_create_batch(out, 1, m, p, stream);
}

void sw_destroy(sw_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->s);
  delete c;
}

sw_status sw_counts(const sw_ctx* c, int64_t* n_cells, int64_t* n_vol, int64_t* n_dofs) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (n_cells) *n_cells = c->K;
  if (n_vol) *n_vol = c->nvol + c->nvv;
  if (n_dofs) *n_dofs = (int64_t)c->K * c->NP;
  return SW_OK;
}

sw_status sw_node_coords(const sw_ctx* c, double* xy) {
  if (!c || !xy) return fail(SW_EINVAL, "NULL argument");
  for (const auto& L : c->lv) {
    for (int cl = 0; cl < L.ncell; ++cl) {
      const int k = L.cell0 + cl;
      const double dx = c->cdx[k], x0 = c->mx0[c->cmem[k]], y0 = c->my0[c->cmem[k]];
      double* o = xy + 2 * (L.off + (size_t)cl * L.S * L.S);
      for (int b = 0; b < L.S; ++b)
        for (int a = 0; a < L.S; ++a) {
          o[2 * (b * L.S + a) + 0] = x0 + (c->ci[k] + L.xh[a]) * dx;
          o[2 * (b * L.S + a) + 1] = y0 + (c->cj[k] + L.xh[b]) * dx;
        }
      if (c->nv > 0) {
        const int nv = c->nv;
        double* ov = xy + 2 * (L.voff + (size_t)cl * nv * nv);
        for (int b = 0; b < nv; ++b)
          for (int a = 0; a < nv; ++a) {
            ov[2 * (b * nv + a) + 0] = x0 + (c->ci[k] + L.xv[a]) * dx;
            ov[2 * (b * nv + a) + 1] = y0 + (c->cj[k] + L.xv[b]) * dx;
          }
      }
    }
  }
  return SW_OK;
}

sw_status sw_locate_points(const sw_ctx* c, int32_t member, int32_t n, const double* xy, int32_t* cell,
                           double* phi) {
  if (!c || (n > 0 && (!xy || !cell || !phi))) return fail(SW_EINVAL, "NULL argument");
  if (member < 0 || member >= c->M) return fail(SW_EINVAL, "member index out of range");
  std::vector<double> xi, wb;
  gll(c->N1, xi, wb);
  for (int g = 0; g < n; ++g) {
    const double x = xy[2 * g], y = xy[2 * g + 1];
    int found = -1;
    double rx = 0.0, ry = 0.0;
    for (int k = 0; k < c->K && found < 0; ++k) {
      if (c->cmem[k] != member) continue;
      const double dx = c->cdx[k];
      const double xl = c->mx0[member] + c->ci[k] * dx, yl = c->my0[member] + c->cj[k] * dx;
      if (x >= xl && x < xl + dx && y >= yl && y < yl + dx) {
        found = k;
        rx = (x - xl) / dx;
        ry = (y - yl) / dx;
      }
    }
    if (found < 0) return fail(SW_EINVAL, "point " + std::to_string(g) + " lies outside the member's mesh");
    cell[g] = found;
    for (int jy = 0; jy < c->N1; ++jy)
      for (int jx = 0; jx < c->N1; ++jx) phi[(size_t)g * c->NP + jy * c->N1 + jx] = lag(xi, jx, rx) * lag(xi, jy, ry);
  }
  return SW_OK;
}

sw_status sw_boundary_nodes(const sw_ctx* c, int64_t* n_nodes, double* xy, int32_t* member) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (n_nodes) *n_nodes = c->ng;
  if (!xy && !member) return SW_OK;
  std::vector<int> fA(c->F), meta(c->F);
  if (hipMemcpy(fA.data(), c->d_fA, c->F * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(meta.data(), c->d_meta, c->F * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(SW_EHIP, "hipMemcpy of the face list failed");
  int64_t o = 0;
  for (int f : c->gface) {
    const int k = fA[f], side = meta[f] & 3, m = c->cmem[k];
    const LevelH& L = c->lv[c->lev[k]];
    const double dx = c->cdx[k];
    for (int al = 0; al < L.S; ++al, ++o) {
      // face nodes in the order of the side's rule (ascending along the face)
      const double X = side == 0 ? 0.0 : side == 1 ? 1.0 : L.xh[al];
      const double Y = side == 2 ? 0.0 : side == 3 ? 1.0 : L.xh[al];
      if (xy) {
        xy[2 * o + 0] = c->mx0[m] + (c->ci[k] + X) * dx;
        xy[2 * o + 1] = c->my0[m] + (c->cj[k] + Y) * dx;
      }
      if (member) member[o] = m;
    }
  }
  return SW_OK;
}

sw_status sw_set_boundary_state(sw_ctx* c, const double* ghost) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (c->ng == 0) return fail(SW_EINVAL, "the mesh has no state or discharge side");
  if (!ghost) return fail(SW_EINVAL, "ghost must be non-NULL");
  const size_t n = (size_t)4 * c->ng;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->s, ghost, c->d_ghost, n);
  HIPCHK(hipGetLastError());
  c->ghost_set = true;
  c->start_ready = false;
  return SW_OK;
}

sw_status sw_cell_map(const sw_ctx* c, int32_t* member, int32_t* local) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  for (int k = 0; k < c->K; ++k) {
    if (member) member[k] = c->cmem[k];
    if (local) local[k] = c->cloc[k];
  }
  return SW_OK;
}

sw_status sw_dof_coords(const sw_ctx* c, double* xy) {
  if (!c || !xy) return fail(SW_EINVAL, "NULL argument");
  std::vector<double> xi, wb;
  gll(c->N1, xi, wb);
  for (int k = 0; k < c->K; ++k) {
    const double dx = c->cdx[k], x0 = c->mx0[c->cmem[k]], y0 = c->my0[c->cmem[k]];
    for (int jy = 0; jy < c->N1; ++jy)
      for (int jx = 0; jx < c->N1; ++jx) {
        const size_t q = (size_t)k * c->NP + jy * c->N1 + jx;
        xy[2 * q + 0] = x0 + (c->ci[k] + xi[jx]) * dx;
        xy[2 * q + 1] = y0 + (c->cj[k] + xi[jy]) * dx;
      }
  }
  return SW_OK;
}

sw_status sw_set_bathymetry(sw_ctx* c, const double* b) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  sw_status st = check_ptr(b, "b");
  if (st != SW_OK) return st;
  const int64_t nb = c->nvol + c->nvv;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, c->s, b, c->d_braw, (size_t)nb);
  HIPCHK(hipGetLastError());
  c->bathy_set = true;
  return rebake(c);
}

sw_status sw_set_bed_offset(sw_ctx* c, const double* db) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  sw_status st = check_ptr(db, "db");
  if (st != SW_OK) return st;
  hipLaunchKernelGGL(k_copy, dim3((c->K + 255) / 256), dim3(256), 0, c->s, db, c->d_db, (size_t)c->K);
  HIPCHK(hipGetLastError());
  if (!c->bathy_set) return SW_OK;
  return rebake(c);
}

sw_status sw_set_manning(sw_ctx* c, const double* n) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  sw_status st = check_ptr(n, "n");
  if (st != SW_OK) return st;
  hipLaunchKernelGGL(k_copy, dim3((c->K + 255) / 256), dim3(256), 0, c->s, n, c->d_nman, (size_t)c->K);
  HIPCHK(hipGetLastError());
  c->start_ready = false;
  return SW_OK;
}

sw_status sw_set_state(sw_ctx* c, const double* eta, const double* qx, const double* qy, const double* tr) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (!eta || !qx || !qy) return fail(SW_EINVAL, "eta, qx, qy must be non-NULL");
  const size_t n = (size_t)c->K * c->NP;
  const unsigned nb = (unsigned)((n + 255) / 256);
  const double* src[4] = {eta, qx, qy, tr};
  for (int q = 0; q < 4; ++q) {
    if (src[q]) hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, c->s, src[q], c->d_sn[q], n);
    else hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, c->s, c->d_sn[q], n, 0.0);
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_fill8, dim3((c->K + 255) / 256), dim3(256), 0, c->s, c->d_flag, (size_t)c->K,
                     (int8_t)c->r);
  HIPCHK(hipGetLastError());
  c->stage_done = 0;
  c->start_ready = false;
  return SW_OK;
}

sw_status sw_get_state(const sw_ctx* c, double* eta, double* qx, double* qy, double* tr) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  const size_t n = (size_t)c->K * c->NP;
  const unsigned nb = (unsigned)((n + 255) / 256);
  double* dst[4] = {eta, qx, qy, tr};
  for (int q = 0; q < 4; ++q) {
    if (!dst[q]) continue;
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, c->s, c->d_sn[q], dst[q], n);
    HIPCHK(hipGetLastError());
  }
  return SW_OK;
}

sw_status sw_init_lake_at_rest(sw_ctx* c, const double* eta) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  sw_status st = check_ptr(eta, "eta");
  if (st != SW_OK) return st;
  if ((st = need_bathy(c)) != SW_OK) return st;
  for (auto& L : c->lv) {
    if (L.ncell == 0) continue;
    hipLaunchKernelGGL(k_lake, dim3((L.ncell + 127) / 128), dim3(128), 0, c->s, L.tabs, L.cell0, L.ncell, L.off,
                       c->N1, c->d_zb, c->d_zmax, eta, c->d_sn[0], c->d_sn[1], c->d_sn[2]);
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_fill8, dim3((c->K + 255) / 256), dim3(256), 0, c->s, c->d_flag, (size_t)c->K,
                     (int8_t)c->r);
  HIPCHK(hipGetLastError());
  c->stage_done = 0;
  c->start_ready = false;
  return SW_OK;
}

sw_status sw_set_time(sw_ctx* c, double t) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  hipLaunchKernelGGL(k_fill_n, dim3((c->M + 255) / 256), dim3(256), 0, c->s, c->d_mt, c->M, t);
  HIPCHK(hipGetLastError());
  return SW_OK;
}

sw_status sw_set_tide(sw_ctx* c, double amplitude, double period, double phase, double c_inflow) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (!(std::fabs(amplitude) < 1e300) || !(std::fabs(period) < 1e300) || period == 0.0 ||
      !(std::fabs(phase) < 1e300) || !(std::fabs(c_inflow) < 1e300))
    return fail(SW_EINVAL, "tide data must be finite with a non-zero period");
  if (c->stage_done != 0) return fail(SW_EINVAL, "sw_set_tide cannot run inside an open step");
  std::vector<double> td(4 * (size_t)c->M);
  for (int m = 0; m < c->M; ++m) {
    td[4 * m + 0] = amplitude;
    td[4 * m + 1] = period;
    td[4 * m + 2] = phase;
    td[4 * m + 3] = c_inflow;
  }
  HIPCHK(hipMemcpyAsync(c->d_mtide, td.data(), td.size() * sizeof(double), hipMemcpyHostToDevice, c->s));
  HIPCHK(hipStreamSynchronize(c->s));   // the host vector goes out of scope
  c->p.tide_amp = amplitude;
  c->p.tide_period = period;
  c->p.tide_phase = phase;
  c->p.tide_c_in = c_inflow;
  c->start_ready = false;
  return SW_OK;
}

namespace {
// The operator evaluation's own device scratch: the residual slot that the
// volume and face kernels accumulate into (res, slot `slot`), the members'
// boundary time (mt), the per-face time-step bounds (fdt), the chunk partials
// of their reduction (part) and the per-member bound (mtmp).
struct ApplyBufs {
  double* res;
  int slot;
  double* mt;
  double* fdt;
  double* part;
  double* mtmp;
};

sw_status apply_impl(sw_ctx* c, const double* eta, const double* qx, const double* qy, const double* tr, double t,
                     double* F, double* Gx, double* Gy, double* R, double* dtb, const ApplyBufs& b) {
  // the helpers below read the context's buffers: point them at b for the
  // launches of this call (kernel arguments are taken at launch)
  struct Swap {
    sw_ctx* c;
    double *res, *fdt, *part;
    ~Swap() {
      c->d_res = res;
      c->d_fdt = fdt;
      c->d_part = part;
    }
  } keep{c, c->d_res, c->d_fdt, c->d_part};
  c->d_res = b.res;
  c->d_fdt = b.fdt;
  c->d_part = b.part;
  sw_status st;
  // the elevation boundary is evaluated at t (stage offset 0)
  hipLaunchKernelGGL(k_fill_n, dim3((c->M + 255) / 256), dim3(256), 0, c->s, b.mt, c->M, t);
  HIPCHK(hipGetLastError());
  for (auto& L : c->lv) {
    StageArgs a = stage_args(c, L);
    a.imex = 0;   // the whole residual, friction included
    a.in[0] = eta;
    a.in[1] = qx;
    a.in[2] = qy;
    a.in[3] = c->p.tracer ? tr : nullptr;
    a.slot = b.slot;
    HIPCHK(launch_stage(c->r, L.P, M_APPLY, a, L.nblk, c->s));
  }
  const double* st4[4] = {eta, qx, qy, c->p.tracer ? tr : eta};
  if ((st = faces(c, st4, 0.0, b.slot, b.mt)) != SW_OK) return st;
  for (auto& L : c->lv) {
    StageArgs a = stage_args(c, L);
    a.slot = b.slot;
    a.out[0] = F;
    a.out[1] = Gx;
    a.out[2] = Gy;
    a.out[3] = c->p.tracer ? R : nullptr;
    HIPCHK(launch_stage(c->r, L.P, M_FOLD, a, L.nblk, c->s));
  }
  if (dtb) {
    // bare positivity bound, minimum over the members
    if ((st = reduce_dt(c, nullptr, b.mtmp)) != SW_OK) return st;
    hipLaunchKernelGGL(k_min_all, dim3(1), dim3(256), 0, c->s, b.mtmp, c->M, dtb);
    HIPCHK(hipGetLastError());
  }
  return SW_OK;
}

sw_status apply_checks(sw_ctx* c, const double* eta, const double* qx, const double* qy, const double* tr, double* F,
                       double* Gx, double* Gy, double* R) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (!eta || !qx || !qy || !F || !Gx || !Gy) return fail(SW_EINVAL, "state and residual pointers must be non-NULL");
  if (c->p.tracer && (!tr || !R)) return fail(SW_EINVAL, "tracer and R are required with a tracer");
  sw_status st = need_inputs(c);
  if (st != SW_OK) return st;
  if (c->stage_done != 0) return fail(SW_EINVAL, "sw_apply_operator cannot run inside an open step");
  return SW_OK;
}
}  // namespace

sw_status sw_apply_operator(sw_ctx* c, const double* eta, const double* qx, const double* qy, const double* tr,
                            double t, double* F, double* Gx, double* Gy, double* R, double* dtb) {
  sw_status st = apply_checks(c, eta, qx, qy, tr, F, Gx, Gy, R);
  if (st != SW_OK) return st;
  const ApplyBufs b{c->d_res, kApplySlot, c->d_mt_apply, c->d_fdt, c->d_part, c->d_mtmp};
  if ((st = apply_impl(c, eta, qx, qy, tr, t, F, Gx, Gy, R, dtb, b)) != SW_OK) return st;
  c->start_ready = false;   // the apply slot does not disturb the step's data, but stay safe
  return SW_OK;
}

sw_status sw_apply_operator_noalloc(sw_ctx* c, const double* eta, const double* qx, const double* qy,
                                    const double* tr, double t, double* F, double* Gx, double* Gy, double* R,
                                    double* dtb) {
  sw_status st = apply_checks(c, eta, qx, qy, tr, F, Gx, Gy, R);
  if (st != SW_OK) return st;
  double* base = scratch_address(c->dev);
  if (!base) return fail(SW_EINVAL, "the device scratch of this context's device was not set up by sw_create");
  // layout, each part rounded up to 32 doubles (256 bytes): one residual slot,
  // member times, face bounds, chunk partials, member bounds
  const size_t KN = (size_t)c->K * c->NP;
  auto up = [](size_t n) { return (n + 31) / 32 * 32; };
  const size_t nres = up(4 * KN), nmt = up((size_t)c->M), nfdt = up((size_t)c->F),
               npart = up((size_t)std::max(c->nfch, c->ncch) * D_NSLOT), nmtmp = up((size_t)c->M);
  const size_t need = nres + nmt + nfdt + npart + nmtmp;
  if (need > kScratchDoubles)
    return fail(SW_EINVAL, "sw_apply_operator_noalloc: this context needs " + std::to_string(need) +
                               " doubles of device scratch, more than the library's fixed " +
                               std::to_string(kScratchDoubles) + " (use sw_apply_operator)");
  // every word a launch reads is written earlier in the same call (volume
  // kernel before the faces, face bounds before their reduction), so nothing
  // left by a previous call is read
  const ApplyBufs b{base, 0, base + nres, base + nres + nmt, base + nres + nmt + nfdt,
                    base + nres + nmt + nfdt + npart};
  return apply_impl(c, eta, qx, qy, tr, t, F, Gx, Gy, R, dtb, b);
}

sw_status sw_step_begin(sw_ctx* c, double dt) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  sw_status st = need_inputs(c);
  if (st != SW_OK) return st;
  if (c->stage_done != 0) return fail(SW_EINVAL, "a step is already open (call sw_rk_stage / sw_step_end)");
  c->fixed_dt = dt > 0.0;
  if (c->fixed_dt) {
    hipLaunchKernelGGL(k_fill_n, dim3((c->M + 255) / 256), dim3(256), 0, c->s, c->d_mdt, c->M, dt);
    HIPCHK(hipGetLastError());
  }
  // degree adaptation, H(zeta^n) and stage-1 volume terms (already in place after
  // a previous step's final kernel)
  if (!c->start_ready || (c->start_replay && !c->replaying))
    if ((st = elements(c, F_START, M_START, -1, 0, 0, nullptr, 0, 0)) != SW_OK) return st;
  c->start_replay = false;
  const double* stn[4] = {c->d_sn[0], c->d_sn[1], c->d_sn[2], c->d_sn[3]};
  if ((st = faces(c, stn, c->c[0], 0)) != SW_OK) return st;
  if (!c->fixed_dt)
    if ((st = reduce_dt(c, c->d_mcfl, c->d_mdt)) != SW_OK) return st;
  c->start_ready = false;
  c->stage_done = 1;
  return SW_OK;
}

sw_status sw_rk_stage(sw_ctx* c, int32_t l) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (l < 2 || l > c->ns) return fail(SW_EINVAL, "stage index out of range");
  if (c->stage_done != l - 1) return fail(SW_EINVAL, "stages must be taken in order after sw_step_begin");
  double coef[4], coeft[4];
  for (int m = 0; m < 4; ++m) {
    coef[m] = m < l - 1 ? c->A[l - 1][m] : 0.0;
    coeft[m] = m < l - 1 ? c->At[l - 1][m] : 0.0;
  }
  // (IMEX: the friction matrix of the previous stage is the one its volume pass stored)
  sw_status st = elements(c, F_STAGE, M_STAGE, -1, l - 1, l - 1, coef, l == 2 ? 1 : 0, 1, coeft,
                          c->At[l - 1][l - 1]);
  if (st != SW_OK) return st;
  const double* sts[4] = {c->d_ss[0], c->d_ss[1], c->d_ss[2], c->d_ss[3]};
  if ((st = faces(c, sts, c->c[l - 1], l - 1)) != SW_OK) return st;
  c->stage_done = l;
  return SW_OK;
}

}  // extern "C"

namespace {

// End of a step after the final combination's launches: per-member
// diagnostics (two-level segmented reduction), each member's time advanced.
sw_status step_end_finish(sw_ctx* c) {
  hipLaunchKernelGGL(k_diag_part_seg, dim3(c->ncch), dim3(256), 0, c->s, c->d_cdiag, c->d_flag, c->d_cch,
                     c->d_part);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_diag_seg, dim3(c->M), dim3(256), 0, c->s, c->d_part, c->d_cch_m0, c->d_mdiag, c->d_mt,
                     c->d_mdt);
  HIPCHK(hipGetLastError());
  c->stage_done = 0;
  c->start_ready = true;
  c->start_replay = c->rp[0] != nullptr;
  ++c->nstep;
  return SW_OK;
}

}  // namespace

extern "C" {

sw_status sw_step_end(sw_ctx* c) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (c->stage_done != c->ns) return fail(SW_EINVAL, "all stages must be taken before sw_step_end");
  // final combination; the same pass prepares the next step's start (slot 0)
  // (IMEX: explicit, the implicit weights b~ = b)
  sw_status st = elements(c, F_FINAL, M_FINAL, M_START, 0, c->ns, c->b, c->ns == 1 ? 1 : 0, 2, c->b);
  if (st != SW_OK) return st;
  return step_end_finish(c);
}

sw_status sw_step(sw_ctx* c, double dt) {
  sw_status st = sw_step_begin(c, dt);
  if (st != SW_OK) return st;
  for (int l = 2; l <= c->ns; ++l)
    if ((st = sw_rk_stage(c, l)) != SW_OK) return st;
  return sw_step_end(c);
}

sw_status sw_step_record(sw_ctx* c, double dt, double* stages, double* end) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (!stages) return fail(SW_EINVAL, "stages must be non-NULL");
  if (!(dt > 0.0)) return fail(SW_EINVAL, "sw_step_record needs a fixed dt > 0");
  const size_t KN = (size_t)c->K * c->NP;
  const unsigned nb = (unsigned)((KN + 255) / 256);
  auto save = [&](double* const* src, int l) -> sw_status {
    for (int f = 0; f < 3; ++f) {
      hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, c->s, src[f], stages + ((size_t)l * 3 + f) * KN, KN);
      HIPCHK(hipGetLastError());
    }
    return SW_OK;
  };
  sw_status st = save(c->d_sn, 0);
  if (st != SW_OK) return st;
  if ((st = sw_step_begin(c, dt)) != SW_OK) return st;
  for (int l = 2; l <= c->ns; ++l) {
    // the stage's kernels write its flow straight into the record (every
    // cell's stage state is written by the stage, and read only within it)
    double* own[3];
    for (int f = 0; f < 3; ++f) {
      own[f] = c->d_ss[f];
      c->d_ss[f] = stages + ((size_t)(l - 1) * 3 + f) * KN;
    }
    st = sw_rk_stage(c, l);
    for (int f = 0; f < 3; ++f) c->d_ss[f] = own[f];
    if (st != SW_OK) return st;
  }
  const size_t KN3 = KN;
  for (int f = 0; f < 3; ++f) c->rec[f] = end ? end + f * KN3 : nullptr;
  st = sw_step_end(c);
  for (int f = 0; f < 3; ++f) c->rec[f] = nullptr;
  return st;
}

sw_status sw_tracer_step(sw_ctx* c, const double* stages, const double* end, double dt) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (!c->p.tracer) return fail(SW_EINVAL, "sw_tracer_step needs a context with a tracer");
  if (!stages || !end) return fail(SW_EINVAL, "stages and end must be non-NULL");
  if (!(dt > 0.0)) return fail(SW_EINVAL, "sw_tracer_step needs the recorded step's dt > 0");
  const size_t KN = (size_t)c->K * c->NP;
  auto point = [&](const double* base) {
    for (int f = 0; f < 3; ++f) c->rp[f] = base ? base + f * KN : nullptr;
  };
  point(nullptr);
  c->replaying = true;
  sw_status st = sw_step_begin(c, dt);
  for (int l = 2; l <= c->ns && st == SW_OK; ++l) {
    point(stages + (size_t)(l - 1) * 3 * KN);
    st = sw_rk_stage(c, l);
  }
  if (st == SW_OK) {
    point(end);
    st = sw_step_end(c);
  }
  point(nullptr);
  c->replaying = false;
  return st;
}

}  // extern "C"

namespace {

sw_status check_tracer_list(const sw_ctx* flow, int32_t n, sw_ctx* const* tracers, double dt) {
  if (!flow) return fail(SW_EINVAL, "NULL flow context");
  if (n < 0 || (n > 0 && !tracers)) return fail(SW_EINVAL, "bad tracer context list");
  if (!(dt > 0.0)) return fail(SW_EINVAL, "sw_step_tracers needs a fixed dt > 0");
  for (int i = 0; i < n; ++i) {
    const sw_ctx* t = tracers[i];
    if (!t || t == flow) return fail(SW_EINVAL, "tracer context " + std::to_string(i) + " is NULL or the flow's");
    if (!t->p.tracer) return fail(SW_EINVAL, "tracer context " + std::to_string(i) + " has no tracer");
    if (t->K != flow->K || t->NP != flow->NP || t->ns != flow->ns || t->M != flow->M || t->lev != flow->lev ||
        t->ci != flow->ci || t->cj != flow->cj || t->cdx != flow->cdx || t->dev != flow->dev)
      return fail(SW_EINVAL, "tracer context " + std::to_string(i) + ": mesh, degree or scheme differ from the flow's");
  }
  return SW_OK;
}

// Records one step of the flow context with the fixed dt: the flow of every
// stage and of the step's end into the context's record buffer.
sw_status record_flow(sw_ctx* flow, double dt, double** stages, double** end) {
  const size_t KN = (size_t)flow->K * flow->NP;
  sw_status st = SW_OK;
  if (!flow->d_trec && (st = flow->alloc(&flow->d_trec, (size_t)(flow->ns + 1) * 3 * KN)) != SW_OK) return st;
  if (!flow->ev_rec) HIPCHK(hipEventCreateWithFlags(&flow->ev_rec, hipEventDisableTiming));
  *stages = flow->d_trec;
  *end = flow->d_trec + (size_t)flow->ns * 3 * KN;
  return sw_step_record(flow, dt, *stages, *end);
}

// R_k of residual slot `slot` += sum_j B_kj int h c_j psi_i for the tracer
// contexts' stage state (stage = the stage state, else the step's state),
// on the flow's stream (every tracer context runs there during the call);
// the contexts carry the same flow and bathymetry, so the depth is the first
// context's
sw_status add_reactions(sw_ctx* const* tr, int n, const double* B, int slot, bool stage) {
  sw_ctx* c0 = tr[0];
  const size_t KN = (size_t)c0->K * c0->NP;
  for (const auto& L : c0->lv) {
    const LevelTabs& t = c0->nv > 0 ? L.vtabs : L.tabs;
    ReactArgs a{};
    a.l = t.l;
    a.w = t.w;
    a.n = t.S;
    a.N1 = c0->N1;
    a.cell0 = L.cell0;
    a.ncell = L.ncell;
    a.M = n;
    a.cdx = c0->d_cdx;
    a.z = stage ? c0->d_ss[0] : c0->d_sn[0];
    a.zb = c0->d_zb + (c0->nv > 0 ? L.voff : L.off);
    for (int j = 0; j < n; ++j) {
      const sw_ctx* c = tr[j];
      a.c[j] = stage ? c->d_ss[3] : c->d_sn[3];
      a.res[j] = c->d_res + ((size_t)slot * 4 + 3) * KN;
    }
    for (int i = 0; i < n * n; ++i) a.B[i] = B[i];
    sw_ctx::Scope sc(tr[0], 7, 1);
    HIPCHK(launch_react(c0->r, a, c0->s));
  }
  return SW_OK;
}

// One replayed stage l of the tracer contexts tr[0..n), whose flow pointers
// name the record's stage: on the sample rule, one launch of the
// multi-tracer kernel per level and group of at most kMaxReact contexts (the
// matrix H(zeta^(l)) factorised once per cell for the group), then each
// context's tracer face terms; otherwise each context's own sw_rk_stage.
sw_status stage_tracers(sw_ctx* const* tr, int n, int l) {
  sw_ctx* c0 = tr[0];
  if (c0->nv > 0 || c0->rp[0] == nullptr) {
    for (int i = 0; i < n; ++i) {
      sw_status st = sw_rk_stage(tr[i], l);
      if (st != SW_OK) return st;
    }
    return SW_OK;
  }
  if (l < 2 || l > c0->ns) return fail(SW_EINVAL, "stage index out of range");
  for (int i = 0; i < n; ++i)
    if (tr[i]->stage_done != l - 1) return fail(SW_EINVAL, "stages must be taken in order after sw_step_begin");
  double coef[4];
  for (int m = 0; m < 4; ++m) coef[m] = m < l - 1 ? c0->A[l - 1][m] : 0.0;
  for (int g0 = 0; g0 < n; g0 += kMaxReact) {
    const int gn = std::min(kMaxReact, n - g0);
    sw_ctx* g = tr[g0];
    for (const auto& L : g->lv) {
      StageArgs a = stage_args(g, L);
      a.slot = l - 1;
      a.nterm = l - 1;
      for (int m = 0; m < 4; ++m) a.a[m] = coef[m];
      a.diag_init = l == 2 ? 1 : 0;
      a.need = nullptr;   // every cell
      TrcSet ts{};
      ts.M = gn;
      for (int j = 0; j < gn; ++j) {
        const sw_ctx* c = tr[g0 + j];
        ts.res[j] = c->d_res;
        ts.cn[j] = c->d_cn;
        ts.c0[j] = c->d_sn[3];
        for (int f = 0; f < 4; ++f) ts.ss[j][f] = c->d_ss[f];
        ts.cdiag[j] = c->d_cdiag;
        ts.tnu[j] = c->p.tracer_diff * c->p.tracer_strain / (double)(c->r * c->r);
        ts.tkap[j] = c->p.tracer_decay;
      }
      sw_ctx::Scope sc(g, 5, 1);
      HIPCHK(launch_trc_multi(g->r, L.P, F_STAGE, a, ts, L.nblk, g->s));
    }
  }
  for (int i = 0; i < n; ++i) {
    sw_ctx* c = tr[i];
    const double* sts[4] = {c->d_ss[0], c->d_ss[1], c->d_ss[2], c->d_ss[3]};
    sw_status st = faces(c, sts, c->c[l - 1], l - 1);
    if (st != SW_OK) return st;
    c->stage_done = l;
  }
  return SW_OK;
}

// One step of the flow context recorded, then the tracer contexts stepped
// stage by stage together over the record on the flow's stream (after their
// earlier work; their streams wait for the call's launches), with the
// reactions react (n x n, or NULL: none) added after each stage's residuals.
sw_status final_tracers(sw_ctx* const* tr, int n);

sw_status step_tracers_impl(sw_ctx* flow, int n, sw_ctx* const* tracers, const double* react, double dt) {
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < i; ++j)
      if (tracers[i] == tracers[j]) return fail(SW_EINVAL, "tracer context " + std::to_string(i) + " is listed twice");
    // one launch steps several contexts: one quadrature and one degree rule
    const sw_ctx* t = tracers[i];
    if (t->nv != tracers[0]->nv)
      return fail(SW_EINVAL, "tracer context " + std::to_string(i) + ": quadrature differs from the first context's");
    if (t->p.h_lim != tracers[0]->p.h_lim || (t->p.adapt_degree != 0) != (tracers[0]->p.adapt_degree != 0))
      return fail(SW_EINVAL, "tracer context " + std::to_string(i) + ": degree adaptation differs from the first context's");
  }
  double *stages = nullptr, *end = nullptr;
  sw_status st = record_flow(flow, dt, &stages, &end);
  if (st != SW_OK || n == 0) return st;
  std::vector<hipStream_t> own(n);
  for (int i = 0; i < n; ++i) {
    sw_ctx* t = tracers[i];
    if (t->s != flow->s) {
      if (!t->ev_rec) HIPCHK(hipEventCreateWithFlags(&t->ev_rec, hipEventDisableTiming));
      HIPCHK(hipEventRecord(t->ev_rec, t->s));
      HIPCHK(hipStreamWaitEvent(flow->s, t->ev_rec, 0));
    }
  }
  for (int i = 0; i < n; ++i) {
    own[i] = ctx_swap_stream(tracers[i], flow->s);
    tracers[i]->replaying = true;
  }
  const size_t KN = (size_t)flow->K * flow->NP;
  auto point = [&](sw_ctx* t, const double* base) {
    for (int f = 0; f < 3; ++f) t->rp[f] = base ? base + f * KN : nullptr;
  };
  // stage by stage over the tracers: a stage's reactions need every tracer's
  // state of that stage, and one launch takes the stage of all of them
  for (int i = 0; i < n && st == SW_OK; ++i) {
    point(tracers[i], nullptr);
    st = sw_step_begin(tracers[i], dt);
  }
  if (st == SW_OK && react) st = add_reactions(tracers, n, react, 0, false);
  for (int l = 2; l <= flow->ns && st == SW_OK; ++l) {
    for (int i = 0; i < n; ++i) point(tracers[i], stages + (size_t)(l - 1) * 3 * KN);
    st = stage_tracers(tracers, n, l);
    if (st == SW_OK && react) st = add_reactions(tracers, n, react, l - 1, true);
  }
  if (st == SW_OK) {
    for (int i = 0; i < n; ++i) point(tracers[i], end);
    st = final_tracers(tracers, n);
  }
  for (int i = 0; i < n; ++i) {
    point(tracers[i], nullptr);
    tracers[i]->replaying = false;
    (void)ctx_swap_stream(tracers[i], own[i]);
  }
  // the tracers' streams wait for what the call launched, also after a failure
  HIPCHK(hipEventRecord(flow->ev_rec, flow->s));
  for (int i = 0; i < n; ++i)
    if (own[i] != flow->s) HIPCHK(hipStreamWaitEvent(own[i], flow->ev_rec, 0));
  return st;
}

// The final combination's StageArgs of one level of a context, as
// sw_step_end forms them.
StageArgs final_args(sw_ctx* c, const LevelH& L) {
  StageArgs a = stage_args(c, L);
  a.slot = 0;
  a.nterm = c->ns;
  for (int m = 0; m < 4; ++m) {
    a.a[m] = c->b[m];
    a.at[m] = c->b[m];
  }
  a.att = 0.0;
  a.diag_init = c->ns == 1 ? 1 : 0;
  return a;
}

// The final combination of the tracer contexts tr[0..n), whose flow pointers
// name the record's end: on the sample rule, each context's degree decision
// on the end flow, then one multi-tracer launch per level and group of at
// most kMaxReact contexts for the cells that keep their degree (H factorised
// once), then each context's general kernel on the others and the end of its
// step; otherwise each context's own sw_step_end.
sw_status final_tracers(sw_ctx* const* tr, int n) {
  sw_ctx* c0 = tr[0];
  if (c0->nv > 0 || c0->rp[0] == nullptr) {
    for (int i = 0; i < n; ++i) {
      sw_status st = sw_step_end(tr[i]);
      if (st != SW_OK) return st;
    }
    return SW_OK;
  }
  for (int i = 0; i < n; ++i)
    if (tr[i]->stage_done != tr[i]->ns) return fail(SW_EINVAL, "all stages must be taken before sw_step_end");
  for (int g0 = 0; g0 < n; g0 += kMaxReact) {
    sw_ctx* c = tr[g0];
    // the step's own degree flags, read by the tracer kernel (the flags of a
    // group's first context stand for the group's)
    hipLaunchKernelGGL(k_copy8, dim3((c->K + 255) / 256), dim3(256), 0, c->s, c->d_flag, c->d_oflag, (size_t)c->K);
    HIPCHK(hipGetLastError());
  }
  // every context holds the same flags and takes the same degree decisions
  // (one flow, one degree rule), so the first context's decision (need[],
  // wflag[]) serves them all
  for (const auto& L : c0->lv) {
    StageArgs d = final_args(c0, L);
    d.need = c0->d_need;
    d.wflag = L.d_wflag;
    HIPCHK(launch_trc_degree(c0->r, L.P, d, L.nblk, c0->s));
  }
  for (int g0 = 0; g0 < n; g0 += kMaxReact) {
    const int gn = std::min(kMaxReact, n - g0);
    sw_ctx* g = tr[g0];
    for (const auto& L : g->lv) {
      StageArgs a = final_args(g, L);
      a.need = c0->d_need;
      TrcSet ts{};
      ts.M = gn;
      for (int j = 0; j < gn; ++j) {
        const sw_ctx* c = tr[g0 + j];
        ts.res[j] = c->d_res;
        ts.cn[j] = c->d_cn;
        ts.c0[j] = c->d_sn[3];
        for (int f = 0; f < 4; ++f) ts.ss[j][f] = c->d_sn[f];
        ts.cdiag[j] = c->d_cdiag;
        ts.tnu[j] = c->p.tracer_diff * c->p.tracer_strain / (double)(c->r * c->r);
        ts.tkap[j] = c->p.tracer_decay;
      }
      sw_ctx::Scope sc(g, 6, 1);
      HIPCHK(launch_trc_multi(g->r, L.P, F_FINAL, a, ts, L.nblk, g->s));
    }
  }
  for (int i = 0; i < n; ++i) {
    sw_ctx* c = tr[i];
    for (size_t l = 0; l < c->lv.size(); ++l) {
      const auto& L = c->lv[l];
      sw_ctx::Scope sc(c, 4, 1);
      StageArgs gk = final_args(c, L);
      gk.need = c0->d_need;
      gk.wflag = c0->lv[l].d_wflag;
      gk.nwave = L.nblk;
      HIPCHK(launch_stage_scan(c->r, L.P, M_FINAL, M_START, gk, std::min(L.nblk, kListGrid), c->s));
    }
    sw_status st = step_end_finish(c);
    if (st != SW_OK) return st;
  }
  return SW_OK;
}

}  // namespace

extern "C" {

sw_status sw_step_tracers_react(sw_ctx* flow, int32_t n, sw_ctx* const* tracers, const double* react, double dt) {
  if (!react) return sw_step_tracers(flow, n, tracers, dt);
  sw_status st = check_tracer_list(flow, n, tracers, dt);
  if (st != SW_OK) return st;
  if (n < 1 || n > kMaxReact)
    return fail(SW_EINVAL, "sw_step_tracers_react couples 1 to " + std::to_string(kMaxReact) + " tracer contexts");
  for (int i = 0; i < n * n; ++i)
    if (!std::isfinite(react[i])) return fail(SW_EINVAL, "reaction matrix entry " + std::to_string(i) + " is not finite");
  return step_tracers_impl(flow, n, tracers, react, dt);
}

sw_status sw_step_tracers(sw_ctx* flow, int32_t n, sw_ctx* const* tracers, double dt) {
  sw_status st = check_tracer_list(flow, n, tracers, dt);
  if (st != SW_OK) return st;
  return step_tracers_impl(flow, n, tracers, nullptr, dt);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Dynamic h-adaptivity (Sec. 3.3 refinement criteria; Sec. 3.4 conservative
// remap, eq:cons-remap, and the mass source Q^n, eq:mass-loss)
// ---------------------------------------------------------------------------
namespace {

// Device buffer from the block cache, returned at scope exit (the call has
// synchronised its stream by then).
struct TmpBuf {
  int dev;
  void* p = nullptr;
  size_t bytes = 0;
  explicit TmpBuf(int d) : dev(d) {}
  hipError_t get(size_t n) {
    bytes = block_bytes(n);
    return cache_alloc(dev, bytes, &p);
  }
  ~TmpBuf() {
    if (p) cache_free(dev, p, bytes);
  }
};

// Bed elevation at every node of the context from its raster, then the depth
// samples, face samples and per-cell tables (as sw_set_bathymetry).
sw_status sample_grid(sw_ctx* c) {
  for (auto& L : c->lv) {
    RasterArgs a{};
    a.g = c->d_grid;
    a.gnx = c->gnx;
    a.gny = c->gny;
    a.gx0 = c->gx0;
    a.gy0 = c->gy0;
    a.gdx = c->gdx;
    a.gdy = c->gdy;
    a.cell0 = L.cell0;
    a.ncell = L.ncell;
    a.n = L.S;
    a.off = L.off;
    a.xh = L.d_xh;
    a.ci = c->d_ci;
    a.cj = c->d_cj;
    a.cdx = c->d_cdx;
    a.cmem = c->d_cmem;
    a.mxy = c->d_mxy;
    a.M = c->M;
    a.braw = c->d_braw;
    HIPCHK(launch_amr_raster(a, c->s));
    if (c->nv > 0) {   // the volume rule's nodes (SW_QUAD_PAPER)
      a.n = c->nv;
      a.off = L.voff;
      a.xh = L.d_xv;
      HIPCHK(launch_amr_raster(a, c->s));
    }
  }
  c->bathy_set = true;
  return rebake(c);
}

// eta_K of every cell at the context's state, at the nodes of the volume
// integrals (those carry bathymetry samples)
sw_status amr_eta(sw_ctx* c, int kind, double* eta) {
  for (auto& L : c->lv) {
    const LevelTabs& t = c->nv > 0 ? L.vtabs : L.tabs;
    AmrEtaArgs a{};
    a.l = t.l;
    a.d = t.d;
    a.n = t.S;
    a.N1 = c->N1;
    a.cell0 = L.cell0;
    a.ncell = L.ncell;
    a.zb = c->d_zb + (c->nv > 0 ? L.voff : L.off);
    a.cdx = c->d_cdx;
    a.z = c->d_sn[0];
    a.qx = c->d_sn[1];
    a.qy = c->d_sn[2];
    a.c = c->d_sn[3];
    a.eps = c->p.eps;
    a.kind = kind;
    a.eta = eta;
    HIPCHK(launch_amr_eta(a, c->s));
  }
  return SW_OK;
}

// Total mass sum_K int h and sum_K int z_b l of the current state on the
// sample rule (synchronises).
sw_status amr_mass(sw_ctx* c, double& mass, double& bathy) {
  TmpBuf b(c->dev);
  HIPCHK(b.get(sizeof(double) * (2 * (size_t)c->K + 2)));
  double* v = (double*)b.p;
  for (auto& L : c->lv) {
    AmrMassArgs a{};
    a.l = L.tabs.l;
    a.w = L.tabs.w;
    a.S = L.S;
    a.N1 = c->N1;
    a.cell0 = L.cell0;
    a.ncell = L.ncell;
    a.zb = c->d_zb + L.off;
    a.cdx = c->d_cdx;
    a.z = c->d_sn[0];
    a.out = v;
    HIPCHK(launch_amr_mass(a, c->s));
  }
  HIPCHK(launch_amr_sum2(v, c->K, v + 2 * (size_t)c->K, c->s));
  double h[2];
  HIPCHK(hipMemcpyAsync(h, v + 2 * (size_t)c->K, sizeof(h), hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  mass = h[0];
  bathy = h[1];
  return SW_OK;
}

// The degree decision and remap that start the next step, if not in place
// (the state the adaptivity acts on; a previous step's final kernel did it).
sw_status ensure_start(sw_ctx* c) {
  if (c->start_ready) return SW_OK;
  sw_status st = elements(c, F_START, M_START, -1, 0, 0, nullptr, 0, 0);
  if (st != SW_OK) return st;
  c->start_ready = true;
  return SW_OK;
}

// The adapted quadtree of one member (see sw_remesh): new leaves in (level,
// j, i) order and, per leaf, the source of its state.
struct AmrPlan {
  std::vector<int> lev, ci, cj, type, src;   // src: 4 per new leaf
  int64_t n_refined = 0, n_coarsened = 0;
};

// One member's leaves (cells sorted by level) and their indicator values.
struct PlanInput {
  int K, nx0, ny0;
  bool perx, pery;
  const int *lev, *ci, *cj;
  const double* cdx;
  const double* eta;
};

AmrPlan amr_plan(const PlanInput& in, double eta_max, const sw_amr_params& ap) {
  struct {
    const int *lev, *ci, *cj;
    const double* cdx;
  } cc{in.lev, in.ci, in.cj, in.cdx}, *c = &cc;
  const int K = in.K;
  const int nx0 = in.nx0, ny0 = in.ny0;
  const bool perx = in.perx, pery = in.pery;
  const double* eta = in.eta;
  // face neighbour position at level L (periodic sides wrap); false outside
  auto neighbour = [&](int L, int i, int j, int di, int dj, int& ni, int& nj) {
    const int nxL = nx0 << L, nyL = ny0 << L;
    ni = i + di;
    nj = j + dj;
    if (ni < 0 || ni >= nxL) {
      if (!perx) return false;
      ni = (ni + nxL) % nxL;
    }
    if (nj < 0 || nj >= nyL) {
      if (!pery) return false;
      nj = (nj + nyL) % nyL;
    }
    return true;
  };
  int maxL = 0;
  for (int k = 0; k < K; ++k) maxL = std::max(maxL, c->lev[k]);
  // levels up to maxL + 1 are looked up (children of refined cells, the cells
  // two levels below a merged parent); the new ones are few and hashed
  LeafIndex idx(nx0, ny0, std::max(maxL + 2, ap.n_max), maxL + 1);
  for (int k = 0; k < K; ++k) idx.set(c->lev[k], c->ci[k], c->cj[k], k);
  std::vector<char> refine(K), coarsen(K), gone(K, 0);
  for (int k = 0; k < K; ++k) {
    refine[k] = eta[k] > ap.theta_r * eta_max && c->lev[k] + 1 < ap.n_max && c->cdx[k] > ap.h_min;
    coarsen[k] = eta[k] < ap.theta_c * eta_max && c->lev[k] > 0 && !refine[k];
  }
  struct Added { int L, i, j; char gone; };
  std::vector<Added> added;
  auto is_leaf = [&](int L, int i, int j) {
    const int v = idx.get(L, i, j);
    return v >= 0 ? !gone[v] : (v <= -2 ? !added[-2 - v].gone : false);
  };
  std::vector<int> queue;   // added leaves whose faces are still to check
  auto split = [&](int L, int i, int j) {
    const int v = idx.get(L, i, j);
    if (v >= 0) gone[v] = 1;
    else added[-2 - v].gone = 1;
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        added.push_back({L + 1, 2 * i + a, 2 * j + b, 0});
        idx.set(L + 1, 2 * i + a, 2 * j + b, -2 - (int)(added.size() - 1));
        queue.push_back((int)added.size() - 1);
      }
  };
  for (int k = 0; k < K; ++k)
    if (refine[k]) split(c->lev[k], c->ci[k], c->cj[k]);
  // 2:1 balance across faces: a new leaf that faces a leaf two or more levels
  // coarser has that leaf refined (only new, finer leaves can create such a
  // pair, so checking each new leaf once reaches the fixed point)
  const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
  for (size_t q = 0; q < queue.size(); ++q) {
    const Added e = added[queue[q]];
    if (e.gone) continue;
    for (int sd = 0; sd < 4; ++sd) {
      int ni, nj;
      if (!neighbour(e.L, e.i, e.j, di[sd], dj[sd], ni, nj)) continue;
      for (int A = e.L - 2; A >= 0; --A)
        if (is_leaf(A, ni >> (e.L - A), nj >> (e.L - A))) {
          split(A, ni >> (e.L - A), nj >> (e.L - A));
          break;
        }
    }
  }
  AmrPlan P;
  for (int k = 0; k < K; ++k) P.n_refined += gone[k];
  // merges of four flagged sibling leaves that keep the balance (decided on
  // the mesh before any merge)
  std::vector<int64_t> parents;
  for (int k = 0; k < K; ++k)
    if (coarsen[k] && !gone[k]) parents.push_back(key(c->lev[k] - 1, c->ci[k] >> 1, c->cj[k] >> 1));
  std::sort(parents.begin(), parents.end());
  parents.erase(std::unique(parents.begin(), parents.end()), parents.end());
  std::vector<std::array<int, 3>> merged;
  for (int64_t pk : parents) {
    const int L = (int)(pk >> 52), pi = (int)((pk >> 26) & ((1 << 26) - 1)), pj = (int)(pk & ((1 << 26) - 1));
    bool ok = true;
    for (int b = 0; b < 2 && ok; ++b)
      for (int a = 0; a < 2 && ok; ++a) {
        const int v = idx.get(L + 1, 2 * pi + a, 2 * pj + b);
        ok = v >= 0 && !gone[v] && coarsen[v];
      }
    for (int sd = 0; sd < 4 && ok; ++sd) {
      int ni, nj;
      if (!neighbour(L, pi, pj, di[sd], dj[sd], ni, nj)) continue;
      for (int t = 0; t < 4 && ok; ++t) {
        int ci, cj;   // level L + 2 cells of the neighbour square along the side
        if (sd == 0) ci = 4 * ni + 3, cj = 4 * nj + t;
        else if (sd == 1) ci = 4 * ni, cj = 4 * nj + t;
        else if (sd == 2) ci = 4 * ni + t, cj = 4 * nj + 3;
        else ci = 4 * ni + t, cj = 4 * nj;
        if (is_leaf(L + 2, ci, cj)) ok = false;
      }
    }
    if (ok) merged.push_back({L, pi, pj});
  }
  for (auto& m : merged) {
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) gone[idx.get(m[0] + 1, 2 * m[1] + a, 2 * m[2] + b)] = 1;
    added.push_back({m[0], m[1], m[2], 0});   // (not entered in idx: no later lookups of it)
  }
  P.n_coarsened = (int64_t)merged.size();
  // new leaves in (level, j, i) order: the kept old cells (in their order when
  // that order is already sorted) merged with the sorted new ones
  auto order = [](int L, int j, int i) { return ((int64_t)L << 52) | ((int64_t)j << 26) | (int64_t)i; };
  bool sorted = true;
  for (int k = 1; k < K && sorted; ++k)
    sorted = order(c->lev[k - 1], c->cj[k - 1], c->ci[k - 1]) < order(c->lev[k], c->cj[k], c->ci[k]);
  std::vector<std::pair<int64_t, int>> newl;   // (order key, old index or -2 - added index)
  for (size_t a = 0; a < added.size(); ++a)
    if (!added[a].gone) newl.push_back({order(added[a].L, added[a].j, added[a].i), -2 - (int)a});
  std::sort(newl.begin(), newl.end());
  std::vector<std::pair<int64_t, int>> all;
  all.reserve((size_t)K + newl.size());
  if (sorted) {
    size_t q = 0;
    for (int k = 0; k < K; ++k) {
      if (gone[k]) continue;
      const int64_t ok = order(c->lev[k], c->cj[k], c->ci[k]);
      while (q < newl.size() && newl[q].first < ok) all.push_back(newl[q++]);
      all.push_back({ok, k});
    }
    while (q < newl.size()) all.push_back(newl[q++]);
  } else {
    for (int k = 0; k < K; ++k)
      if (!gone[k]) all.push_back({order(c->lev[k], c->cj[k], c->ci[k]), k});
    all.insert(all.end(), newl.begin(), newl.end());
    std::sort(all.begin(), all.end());
  }
  const size_t Kn = all.size();
  P.lev.resize(Kn);
  P.ci.resize(Kn);
  P.cj.resize(Kn);
  P.type.resize(Kn);
  P.src.assign(4 * Kn, 0);
  for (size_t n = 0; n < Kn; ++n) {
    const int v = all[n].second;
    int L, i, j;
    if (v >= 0) {
      L = c->lev[v], i = c->ci[v], j = c->cj[v];
      P.type[n] = 0;
      P.src[4 * n] = v;
    } else {
      const Added& e = added[-2 - v];
      L = e.L, i = e.i, j = e.j;
      const int par = L > 0 ? idx.get(L - 1, i >> 1, j >> 1) : -1;
      if (par >= 0 && gone[par]) {   // a child of a refined old cell
        P.type[n] = 1;
        P.src[4 * n] = par;
        P.src[4 * n + 1] = 2 * (j & 1) + (i & 1);
      } else {                       // a parent of four old cells
        P.type[n] = 2;
        for (int b = 0; b < 2; ++b)
          for (int a = 0; a < 2; ++a) {
            const int kd = idx.get(L + 1, 2 * i + a, 2 * j + b);
            P.src[4 * n + 2 * b + a] = kd >= 0 ? kd : -1;
          }
      }
    }
    P.lev[n] = L;
    P.ci[n] = i;
    P.cj[n] = j;
  }
  return P;
}

// Transfer tables of degree r on the unit square: child[s][j][k] = psi_k at
// child s's support point j (s = 2 sy + sx); proj[s][j][k]: the exact-mass L2
// projection's part from child s, parent_j = sum_s sum_k proj[s][j][k] child_s,k.
bool transfer_tables(int r, std::vector<double>& child, std::vector<double>& proj) {
  const int N1 = r + 1, NP = N1 * N1;
  std::vector<double> xi, wb, xg, wg;
  gll(N1, xi, wb);
  gl(N1, xg, wg);
  child.assign((size_t)4 * NP * NP, 0.0);
  proj.assign((size_t)4 * NP * NP, 0.0);
  std::vector<double> Mq((size_t)NP * NP, 0.0);
  for (int i = 0; i < NP; ++i)
    for (int j = 0; j < NP; ++j) {
      double s = 0.0;
      for (int b = 0; b < N1; ++b)
        for (int a = 0; a < N1; ++a)
          s += wg[a] * wg[b] * lag(xi, i % N1, xg[a]) * lag(xi, i / N1, xg[b]) * lag(xi, j % N1, xg[a]) *
               lag(xi, j / N1, xg[b]);
      Mq[(size_t)i * NP + j] = s;
    }
  if (!spd_inverse(Mq, NP)) return false;
  for (int s = 0; s < 4; ++s) {
    const int sx = s & 1, sy = s >> 1;
    double* T = child.data() + (size_t)s * NP * NP;
    for (int j = 0; j < NP; ++j) {
      const double X = 0.5 * (sx + xi[j % N1]), Y = 0.5 * (sy + xi[j / N1]);
      for (int k = 0; k < NP; ++k) T[(size_t)j * NP + k] = lag(xi, k % N1, X) * lag(xi, k / N1, Y);
    }
    std::vector<double> rhs((size_t)NP * NP, 0.0);   // int_child psi_i^parent psi_k^child
    for (int i = 0; i < NP; ++i)
      for (int k = 0; k < NP; ++k) {
        double acc = 0.0;
        for (int b = 0; b < N1; ++b)
          for (int a = 0; a < N1; ++a)
            acc += 0.25 * wg[a] * wg[b] * lag(xi, i % N1, 0.5 * (sx + xg[a])) * lag(xi, i / N1, 0.5 * (sy + xg[b])) *
                   lag(xi, k % N1, xg[a]) * lag(xi, k / N1, xg[b]);
        rhs[(size_t)i * NP + k] = acc;
      }
    double* Pm = proj.data() + (size_t)s * NP * NP;
    for (int j = 0; j < NP; ++j)
      for (int k = 0; k < NP; ++k) {
        double acc = 0.0;
        for (int i = 0; i < NP; ++i) acc += Mq[(size_t)j * NP + i] * rhs[(size_t)i * NP + k];
        Pm[(size_t)j * NP + k] = acc;
      }
  }
  return true;
}

sw_status amr_common_checks(sw_ctx* c) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (c->M != 1) return fail(SW_EINVAL, "mesh adaptivity covers single-member contexts");
  if (c->stage_done != 0) return fail(SW_EINVAL, "mesh adaptivity cannot run inside an open step");
  return need_bathy(c);
}

}  // namespace

extern "C" {

sw_status sw_amr_plan(const sw_mesh_desc* mesh, const double* eta, const sw_amr_params* ap, int32_t cap,
                      int32_t* n_new, int32_t* level, int32_t* i, int32_t* j, int32_t* type, int32_t* src,
                      int64_t* n_refined, int64_t* n_coarsened) {
  if (!mesh || !eta || !ap || !n_new) return fail(SW_EINVAL, "NULL argument to sw_amr_plan");
  const int K = mesh->n_cells;
  if (K < 1 || !mesh->level || !mesh->i || !mesh->j || mesh->nx0 < 1 || mesh->ny0 < 1 || !(mesh->dx0 > 0.0))
    return fail(SW_EINVAL, "bad mesh");
  if (ap->n_max < 1 || ap->n_max > 24) return fail(SW_EINVAL, "n_max must be 1 .. 24");
  std::vector<double> cdx(K);
  std::unordered_set<int64_t> seen;
  seen.reserve((size_t)K * 2);
  for (int k = 0; k < K; ++k) {
    const int L = mesh->level[k];
    if (L < 0 || L > 24 || mesh->i[k] < 0 || mesh->j[k] < 0 || mesh->i[k] >= (mesh->nx0 << L) ||
        mesh->j[k] >= (mesh->ny0 << L))
      return fail(SW_EINVAL, "cell outside the domain");
    if (!seen.insert(key(L, mesh->i[k], mesh->j[k])).second) return fail(SW_EINVAL, "duplicate cell");
    cdx[k] = mesh->dx0 / std::ldexp(1.0, L);
  }
  double eta_max = 0.0;
  for (int k = 0; k < K; ++k) eta_max = std::max(eta_max, eta[k]);
  PlanInput pin{K, mesh->nx0, mesh->ny0, mesh->bc[0] == SW_BC_PERIODIC, mesh->bc[2] == SW_BC_PERIODIC,
                mesh->level, mesh->i, mesh->j, cdx.data(), eta};
  AmrPlan P = amr_plan(pin, eta_max, *ap);
  const int Kn = (int)P.lev.size();
  *n_new = Kn;
  if (n_refined) *n_refined = P.n_refined;
  if (n_coarsened) *n_coarsened = P.n_coarsened;
  if (cap < Kn) return fail(SW_EINVAL, "sw_amr_plan: the new mesh has " + std::to_string(Kn) + " cells, more than cap");
  for (int n = 0; n < Kn; ++n) {
    if (level) level[n] = P.lev[n];
    if (i) i[n] = P.ci[n];
    if (j) j[n] = P.cj[n];
    if (type) type[n] = P.type[n];
    if (src)
      for (int q = 0; q < 4; ++q) src[4 * n + q] = P.src[4 * n + q];
  }
  return SW_OK;
}

sw_status sw_cells(const sw_ctx* c, int32_t* level, int32_t* i, int32_t* j) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  for (int k = 0; k < c->K; ++k) {
    if (level) level[k] = c->lev[k];
    if (i) i[k] = c->ci[k];
    if (j) j[k] = c->cj[k];
  }
  return SW_OK;
}

sw_status sw_set_bed_grid(sw_ctx* c, int32_t nx, int32_t ny, double x0, double y0, double dx, double dy,
                          const double* b) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (!b) return fail(SW_EINVAL, "b is NULL");
  if (nx < 2 || ny < 2 || (int64_t)nx * ny > ((int64_t)1 << 31))
    return fail(SW_EINVAL, "the raster needs 2 <= nx, ny and nx ny <= 2^31");
  if (!(dx > 0.0 && dx < 1e300) || !(dy > 0.0 && dy < 1e300) || !(std::fabs(x0) < 1e300) ||
      !(std::fabs(y0) < 1e300))
    return fail(SW_EINVAL, "raster spacing must be finite and > 0, its origin finite");
  const size_t n = (size_t)nx * ny;
  if (!c->d_grid || (size_t)c->gnx * c->gny != n) {
    if (c->d_grid) {   // the previous raster's memory
      HIPCHK(hipStreamSynchronize(c->s));
      auto it = std::find_if(c->allocs.begin(), c->allocs.end(),
                             [&](const std::pair<void*, size_t>& a) { return a.first == (void*)c->d_grid; });
      if (it != c->allocs.end()) {
        cache_free(c->dev, it->first, it->second);
        c->allocs.erase(it);
      }
      c->d_grid = nullptr;
    }
    sw_status st = c->alloc(&c->d_grid, n);
    if (st != SW_OK) return st;
  }
  HIPCHK(hipMemcpyAsync(c->d_grid, b, n * sizeof(double), hipMemcpyDeviceToDevice, c->s));
  c->gnx = nx;
  c->gny = ny;
  c->gx0 = x0;
  c->gy0 = y0;
  c->gdx = dx;
  c->gdy = dy;
  return sample_grid(c);
}

sw_status sw_amr_indicator(sw_ctx* c, int32_t kind, double* eta) {
  sw_status st = amr_common_checks(c);
  if (st != SW_OK) return st;
  if (!eta) return fail(SW_EINVAL, "eta is NULL");
  if (kind != SW_AMR_VORTICITY && kind != SW_AMR_TRACER_GRAD) return fail(SW_EINVAL, "unknown indicator");
  if (kind == SW_AMR_TRACER_GRAD && !c->p.tracer) return fail(SW_EINVAL, "the tracer indicator needs a tracer");
  if ((st = ensure_start(c)) != SW_OK) return st;
  return amr_eta(c, kind, eta);
}

sw_status sw_remesh(sw_ctx* c, const sw_amr_params* ap, sw_amr_stats* out) {
  sw_status st = amr_common_checks(c);
  if (st != SW_OK) return st;
  if (!ap) return fail(SW_EINVAL, "NULL adaptivity parameters");
  if (ap->indicator != SW_AMR_VORTICITY && ap->indicator != SW_AMR_TRACER_GRAD)
    return fail(SW_EINVAL, "unknown indicator");
  if (ap->indicator == SW_AMR_TRACER_GRAD && !c->p.tracer)
    return fail(SW_EINVAL, "the tracer indicator needs a tracer");
  if (!(ap->theta_r >= 0.0 && ap->theta_r < 1e300) || !(ap->theta_c >= 0.0 && ap->theta_c < 1e300) ||
      !(ap->h_min >= 0.0 && ap->h_min < 1e300))
    return fail(SW_EINVAL, "theta_r, theta_c and h_min must be finite and >= 0");
  if (ap->n_max < 1 || ap->n_max > c->p.n_levels)
    return fail(SW_EINVAL, "n_max must be 1 .. n_levels (params.S gives every level's sample count)");
  if (!c->d_grid) return fail(SW_EINVAL, "sw_remesh samples new cells from the raster of sw_set_bed_grid");
  if ((st = ensure_start(c)) != SW_OK) return st;
  const int K = c->K;
  std::vector<double> eta(K);
  {
    TmpBuf b(c->dev);
    HIPCHK(b.get(sizeof(double) * (size_t)std::max(K, 1)));
    if ((st = amr_eta(c, ap->indicator, (double*)b.p)) != SW_OK) return st;
    HIPCHK(hipMemcpyAsync(eta.data(), b.p, sizeof(double) * K, hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
  }
  double eta_max = 0.0;
  for (double e : eta) eta_max = std::max(eta_max, e);
  sw_amr_stats S{};
  S.n_cells_old = K;
  S.eta_max = eta_max;
  if ((st = amr_mass(c, S.mass_old, S.q_bathy)) != SW_OK) return st;
  const double bathy_old = S.q_bathy;
  PlanInput pin{K, c->mnx0[0], c->mny0[0], c->mbc[0][0] == SW_BC_PERIODIC, c->mbc[0][2] == SW_BC_PERIODIC,
                c->lev.data(), c->ci.data(), c->cj.data(), c->cdx.data(), eta.data()};
  AmrPlan P = amr_plan(pin, eta_max, *ap);
  S.n_refined = P.n_refined;
  S.n_coarsened = P.n_coarsened;
  S.n_cells_new = (int64_t)P.lev.size();
  if (P.n_refined == 0 && P.n_coarsened == 0) {
    S.mass_new = S.mass_old;
    S.q_bathy = 0.0;
    S.boundary_data_kept = c->ghost_set ? 1 : 0;
    if (out) *out = S;
    return SW_OK;
  }
  for (size_t q = 0; q < P.src.size(); ++q)
    if (P.src[q] < 0) return fail(SW_EINVAL, "sw_remesh: a new cell has no source cell");
  std::vector<double> tchild, tproj;
  if (!transfer_tables(c->r, tchild, tproj)) return fail(SW_EINVAL, "sw_remesh: mass matrix not SPD");
  // the context of the new mesh, on the same stream with the same parameters
  sw_mesh_desc md{};
  md.nx0 = c->mnx0[0];
  md.ny0 = c->mny0[0];
  md.x0 = c->mx0[0];
  md.y0 = c->my0[0];
  md.dx0 = c->mdx0[0];
  md.n_cells = (int32_t)P.lev.size();
  md.level = P.lev.data();
  md.i = P.ci.data();
  md.j = P.cj.data();
  for (int sd = 0; sd < 4; ++sd) md.bc[sd] = c->mbc[0][sd];
  sw_ctx* n = nullptr;
  if ((st = create_ctx(&n, 1, &md, &c->p, c->s, true)) != SW_OK) return st;
  auto drop = [&](sw_status e) {
    (void)hipStreamSynchronize(c->s);
    delete n;
    return e;
  };
  const int Kn = n->K, NP = c->NP;
  TmpBuf bt(c->dev), bs(c->dev), btab(c->dev);
  auto d2d = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->s);
  };
  hipError_t e = hipSuccess;
  // member time, time step, tide, CFL number and diagnostics carry over
  if (e == hipSuccess) e = d2d(n->d_mt, c->d_mt, sizeof(double));
  if (e == hipSuccess) e = d2d(n->d_mdt, c->d_mdt, sizeof(double));
  if (e == hipSuccess) e = d2d(n->d_mtide, c->d_mtide, 4 * sizeof(double));
  if (e == hipSuccess) e = d2d(n->d_mcfl, c->d_mcfl, sizeof(double));
  if (e == hipSuccess) e = d2d(n->d_mdiag, c->d_mdiag, kMDiag * sizeof(double));
  if (e == hipSuccess && n->alloc(&n->d_grid, (size_t)c->gnx * c->gny) != SW_OK) e = hipErrorOutOfMemory;
  if (e == hipSuccess) e = d2d(n->d_grid, c->d_grid, sizeof(double) * (size_t)c->gnx * c->gny);
  if (e == hipSuccess) e = bt.get(sizeof(int) * (size_t)Kn);
  if (e == hipSuccess) e = bs.get(sizeof(int) * 4 * (size_t)Kn);
  if (e == hipSuccess) e = btab.get(sizeof(double) * 8 * (size_t)NP * NP);
  if (e == hipSuccess) e = hipMemcpyAsync(bt.p, P.type.data(), sizeof(int) * Kn, hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess) e = hipMemcpyAsync(bs.p, P.src.data(), sizeof(int) * 4 * Kn, hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(btab.p, tchild.data(), sizeof(double) * 4 * NP * NP, hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess)
    e = hipMemcpyAsync((double*)btab.p + 4 * NP * NP, tproj.data(), sizeof(double) * 4 * NP * NP,
                       hipMemcpyHostToDevice, c->s);
  if (e != hipSuccess) return drop(fail(SW_EHIP, std::string("sw_remesh: ") + hipGetErrorString(e)));
  n->gnx = c->gnx;
  n->gny = c->gny;
  n->gx0 = c->gx0;
  n->gy0 = c->gy0;
  n->gdx = c->gdx;
  n->gdy = c->gdy;
  AmrXferArgs x{};
  x.Kn = Kn;
  x.NP = NP;
  x.type = (const int*)bt.p;
  x.src = (const int*)bs.p;
  x.tchild = (const double*)btab.p;
  x.tproj = (const double*)btab.p + 4 * NP * NP;
  for (int f = 0; f < 4; ++f) {
    x.in[f] = c->d_sn[f];
    x.out[f] = n->d_sn[f];
  }
  x.nman_in = c->d_nman;
  x.db_in = c->d_db;
  x.nman_out = n->d_nman;
  x.db_out = n->d_db;
  if ((e = launch_amr_transfer(x, c->s)) != hipSuccess)
    return drop(fail(SW_EHIP, std::string("sw_remesh: ") + hipGetErrorString(e)));
  // the bathymetry of the new cells (with the transferred bed offsets)
  if ((st = sample_grid(n)) != SW_OK) return drop(st);
  // given boundary data carry over when the faces that take them are the
  // same cells' same sides, in the same order
  bool keep = c->ghost_set && c->ng > 0 && n->ng == c->ng && n->gface.size() == c->gface.size();
  for (size_t g = 0; keep && g < c->gface.size(); ++g) {
    const int a = c->gcell[g], b = n->gcell[g];
    keep = c->gside[g] == n->gside[g] && c->lev[a] == n->lev[b] && c->ci[a] == n->ci[b] && c->cj[a] == n->cj[b];
  }
  if (keep) {
    if ((e = d2d(n->d_ghost, c->d_ghost, sizeof(double) * 4 * (size_t)c->ng)) != hipSuccess)
      return drop(fail(SW_EHIP, std::string("sw_remesh: ") + hipGetErrorString(e)));
    n->ghost_set = true;
  }
  S.boundary_data_kept = keep ? 1 : 0;
  double bathy_new = 0.0;
  if ((st = amr_mass(n, S.mass_new, bathy_new)) != SW_OK) return drop(st);
  S.q_bathy = bathy_new - bathy_old;
  n->prof = c->prof;
  n->prof_mask = c->prof_mask;
  n->nstep = c->nstep;
  HIPCHK(hipStreamSynchronize(c->s));
  c->adopt(*n);
  delete n;
  if (out) *out = S;
  return SW_OK;
}

}  // extern "C"

namespace {

VjpArgs vjp_args(sw_ctx* c, const LevelH& L) {
  VjpArgs a{};
  a.t = L.tabs;
  a.cell0 = L.cell0;
  a.ncell = L.ncell;
  a.K = c->K;
  a.zb = c->d_zb + L.off;
  a.nman = c->d_nman;
  a.cdx = c->d_cdx;
  a.err = c->d_err;
  a.g = c->p.g;
  a.eps = c->p.eps;
  a.hlim = c->p.h_lim;
  return a;
}

// face part of the residual VJP for every level and class, then the per-cell
// gather of the bed-offset parts
sw_status vjp_faces(sw_ctx* c, const double* const* u, const double* const* rb, double* const* ub, double tt,
                    double* dbbar) {
  for (auto& L : c->lv)
    for (int k = 0; k < 6; ++k) {
      if (L.cnface[k] == 0) continue;
      VjpFaceArgs a{};
      a.face0 = L.cface0[k];
      a.nface = L.cnface[k];
      a.K = c->K;
      a.S = L.S;
      a.fA = c->d_fA;
      a.fB = c->d_fB;
      a.meta = c->d_meta;
      a.zf = c->d_zf + L.zfoff + (size_t)(L.cface0[k] - L.face0) * 2 * L.S;
      for (int f = 0; f < 3; ++f) {
        a.u[f] = u[f];
        a.rb[f] = rb[f];
        a.ub[f] = ub[f];
      }
      a.fdb = c->d_fdb;
      a.cdx = c->d_cdx;
      a.cmem = c->d_cmem;
      a.fl = L.tabs.fl;
      a.w = L.tabs.w;
      a.mtide = c->d_mtide;
      a.gof = c->d_gof;
      a.ghost = c->d_ghost;
      a.ng = c->ng;
      a.tt = tt;
      a.err = c->d_err;
      a.g = c->p.g;
      a.eps = c->p.eps;
      HIPCHK(launch_vjp_face(c->r, a, L.cfnblk[k], c->s));
    }
  hipLaunchKernelGGL(k_gather_fdb, dim3((c->K + 255) / 256), dim3(256), 0, c->s, c->d_fdb, c->d_cfoff, c->d_cfent,
                     c->K, dbbar);
  HIPCHK(hipGetLastError());
  return SW_OK;
}

}  // namespace

extern "C" {

sw_status sw_vjp_operator(sw_ctx* c, const double* eta, const double* qx, const double* qy, double t,
                          const double* Fb, const double* Gxb, const double* Gyb, double* eta_b, double* qx_b,
                          double* qy_b, double* n_bar, double* db_bar) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (!eta || !qx || !qy || !Fb || !Gxb || !Gyb || !eta_b || !qx_b || !qy_b || !n_bar || !db_bar)
    return fail(SW_EINVAL, "all arrays of sw_vjp_operator must be non-NULL");
  if (c->nv > 0) return fail(SW_EINVAL, "the adjoint covers the sample-rule quadrature, not SW_QUAD_PAPER");
  sw_status st = need_inputs(c);
  if (st != SW_OK) return st;
  const unsigned nbk = (unsigned)((c->K + 255) / 256);
  hipLaunchKernelGGL(k_fill, dim3(nbk), dim3(256), 0, c->s, n_bar, (size_t)c->K, 0.0);
  hipLaunchKernelGGL(k_fill, dim3(nbk), dim3(256), 0, c->s, db_bar, (size_t)c->K, 0.0);
  HIPCHK(hipGetLastError());
  const double* u[3] = {eta, qx, qy};
  const double* rb[3] = {Fb, Gxb, Gyb};
  double* ub[3] = {eta_b, qx_b, qy_b};
  for (auto& L : c->lv) {
    VjpArgs a = vjp_args(c, L);
    for (int f = 0; f < 3; ++f) {
      a.u[f] = u[f];
      a.rin[f] = rb[f];
      a.ub[f] = ub[f];
    }
    a.nbar = n_bar;
    a.dbbar = db_bar;
    HIPCHK(launch_vjp_vol(c->r, L.P, V_OP, a, L.nblk, c->s));
  }
  return vjp_faces(c, u, rb, ub, t, db_bar);
}

sw_status sw_vjp_step(sw_ctx* c, const double* stages, double t, double dt, double* state_bar, double* n_bar,
                      double* db_bar) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (!stages || !state_bar || !n_bar || !db_bar) return fail(SW_EINVAL, "arrays of sw_vjp_step must be non-NULL");
  if (!(dt > 0.0)) return fail(SW_EINVAL, "sw_vjp_step needs the step's fixed dt > 0");
  if (c->p.tracer) return fail(SW_EINVAL, "the step adjoint covers runs without a tracer");
  if (c->imex) return fail(SW_EINVAL, "the step adjoint covers the explicit schemes, not IMEX");
  if (c->nv > 0) return fail(SW_EINVAL, "the adjoint covers the sample-rule quadrature, not SW_QUAD_PAPER");
  if (c->stage_done != 0) return fail(SW_EINVAL, "sw_vjp_step cannot run inside an open step");
  sw_status st = need_inputs(c);
  if (st != SW_OK) return st;
  const size_t KN = (size_t)c->K * c->NP;
  const int ns = c->ns;
  double* sb[3] = {state_bar, state_bar + KN, state_bar + 2 * KN};
  auto slot = [&](int l, int f) { return c->d_res + ((size_t)l * 4 + f) * KN; };
  for (int l = ns; l >= 1; --l) {
    const double* u[3];
    for (int f = 0; f < 3; ++f) u[f] = stages + ((size_t)(l - 1) * 3 + f) * KN;
    double* ub[3] = {slot(l - 1, 0), slot(l - 1, 1), slot(l - 1, 2)};
    const double* rb[3] = {c->d_ss[0], c->d_ss[1], c->d_ss[2]};
    for (auto& L : c->lv) {
      VjpArgs a = vjp_args(c, L);
      for (int f = 0; f < 3; ++f) {
        a.u[f] = u[f];
        a.rbar[f] = c->d_ss[f];
        a.ub[f] = ub[f];
        a.yb[0][f] = sb[f];
      }
      a.yc[0] = c->b[l - 1];
      int ny = 1;
      for (int m = l + 1; m <= ns; ++m, ++ny) {
        for (int f = 0; f < 3; ++f) a.yb[ny][f] = slot(m - 1, f);
        a.yc[ny] = c->A[m - 1][l - 1];
      }
      a.ny = ny;
      a.dt = dt;
      a.nbar = n_bar;
      a.dbbar = db_bar;
      a.check = (l == 1 && c->p.adapt_degree) ? 2 : 1;
      HIPCHK(launch_vjp_vol(c->r, L.P, V_STEP, a, L.nblk, c->s));
    }
    if ((st = vjp_faces(c, u, rb, ub, t + c->c[l - 1] * dt, db_bar)) != SW_OK) return st;
  }
  hipLaunchKernelGGL(k_vjp_combine, dim3((unsigned)((KN + 255) / 256)), dim3(256), 0, c->s, sb[0], sb[1], sb[2],
                     (const double*)c->d_res, ns, KN);
  HIPCHK(hipGetLastError());
  c->start_ready = false;   // the residual slots were used as scratch
  return SW_OK;
}

sw_status sw_run(sw_ctx* c, int32_t n, double dt) {
  for (int i = 0; i < n; ++i) {
    sw_status st = sw_step(c, dt);
    if (st != SW_OK) return st;
  }
  return SW_OK;
}

sw_status sw_sync(sw_ctx* c) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  HIPCHK(hipStreamSynchronize(c->s));
  int err = 0;
  HIPCHK(hipMemcpy(&err, c->d_err, sizeof(int), hipMemcpyDeviceToHost));
  if (err) return fail(SW_EDEVICE, "a kernel reported an invalid index (code " + std::to_string(err) + ")");
  return SW_OK;
}

sw_status sw_set_workgroup(sw_ctx* c, int32_t level, int32_t kernel, int32_t value) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (kernel == 0) {
    if (value != 1 && value != 2 && value != 4) return fail(SW_EINVAL, "wavefronts per workgroup must be 1, 2 or 4");
  } else if (kernel == 1) {
    if (value != 2 && value != 4 && value != 8) return fail(SW_EINVAL, "lanes per face must be 2, 4 or 8");
  } else if (kernel == 2) {
    if (value < -1 || value > 1) return fail(SW_EINVAL, "element order must be -1, 0 or 1");
  } else {
    return fail(SW_EINVAL, "kernel must be 0 (fast element kernel), 1 (face kernel) or 2 (element order)");
  }
  for (auto& L : c->lv)
    if (level < 0 || L.L == level) (kernel == 0 ? L.wpb : kernel == 1 ? L.face_q : L.xorder) = value;
  return SW_OK;
}

sw_status sw_autotune(sw_ctx* c, int32_t steps, double dt, int32_t* wpb_out, int32_t* q_out) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (steps < 1 || steps > 1000) return fail(SW_EINVAL, "steps must be 1..1000");
  sw_status st = need_inputs(c);
  if (st != SW_OK) return st;
  if (c->stage_done != 0) return fail(SW_EINVAL, "sw_autotune cannot run inside an open step");
  // snapshot of everything a step changes that the next step reads
  const size_t KN = (size_t)c->K * c->NP;
  std::vector<void*> keep;
  auto dalloc = [&](size_t bytes) -> void* {
    void* q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) return nullptr;
    keep.push_back(q);
    return q;
  };
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(c->s);
    for (void* q : keep) (void)hipFree(q);
  };
  double* snap = (double*)dalloc(sizeof(double) * (4 * KN + 18 * (size_t)c->M));
  int8_t* sflag = (int8_t*)dalloc((size_t)c->K);
  if (!snap || !sflag) {
    cleanup();
    return fail(SW_ENOMEM, "sw_autotune: no memory for the state snapshot");
  }
  auto copy = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->s);
  };
  hipError_t e = hipSuccess;
  for (int f = 0; f < 4 && e == hipSuccess; ++f) e = copy(snap + f * KN, c->d_sn[f], sizeof(double) * KN);
  if (e == hipSuccess) e = copy(snap + 4 * KN, c->d_mt, sizeof(double) * c->M);
  if (e == hipSuccess) e = copy(snap + 4 * KN + c->M, c->d_mdt, sizeof(double) * c->M);
  if (e == hipSuccess) e = copy(snap + 4 * KN + 2 * c->M, c->d_mdiag, sizeof(double) * kMDiag * c->M);
  if (e == hipSuccess) e = copy(sflag, c->d_flag, (size_t)c->K);
  auto restore = [&]() {
    hipError_t r = hipSuccess;
    for (int f = 0; f < 4 && r == hipSuccess; ++f) r = copy(c->d_sn[f], snap + f * KN, sizeof(double) * KN);
    if (r == hipSuccess) r = copy(c->d_mt, snap + 4 * KN, sizeof(double) * c->M);
    if (r == hipSuccess) r = copy(c->d_mdt, snap + 4 * KN + c->M, sizeof(double) * c->M);
    if (r == hipSuccess) r = copy(c->d_mdiag, snap + 4 * KN + 2 * c->M, sizeof(double) * kMDiag * c->M);
    if (r == hipSuccess) r = copy(c->d_flag, sflag, (size_t)c->K);
    c->start_ready = false;
    c->stage_done = 0;
    return r;
  };
  const int64_t nstep0 = c->nstep;
  const bool prof0 = c->prof;
  c->prof = false;
  hipEvent_t ea = nullptr, eb = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&ea);
  if (e == hipSuccess) e = hipEventCreate(&eb);
  const int wpbs[3] = {1, 2, 4}, qs[3] = {2, 4, 8};
  int bw = c->lv[0].wpb, bq = c->lv[0].face_q, bo = c->lv[0].xorder;
  float best = 1e30f;
  for (int io = 0; io < 2 && e == hipSuccess && st == SW_OK; ++io)
  for (int iw = 0; iw < 3 && e == hipSuccess && st == SW_OK; ++iw)
    for (int iq = 0; iq < 3 && e == hipSuccess && st == SW_OK; ++iq) {
      for (auto& L : c->lv) {
        L.wpb = wpbs[iw];
        L.face_q = qs[iq];
        L.xorder = io;
      }
      if ((e = restore()) != hipSuccess) break;
      if ((st = sw_step(c, dt)) != SW_OK) break;   // start-of-step terms and warm caches
      if ((e = hipEventRecord(ea, c->s)) != hipSuccess) break;
      if ((st = sw_run(c, steps, dt)) != SW_OK) break;
      if ((e = hipEventRecord(eb, c->s)) != hipSuccess) break;
      if ((e = hipEventSynchronize(eb)) != hipSuccess) break;
      float ms = 0.0f;
      if ((e = hipEventElapsedTime(&ms, ea, eb)) != hipSuccess) break;
      if (ms < best) {
        best = ms;
        bw = wpbs[iw];
        bq = qs[iq];
        bo = io;
      }
    }
  for (auto& L : c->lv) {
    L.wpb = bw;
    L.face_q = bq;
    L.xorder = bo;
  }
  if (e == hipSuccess && st == SW_OK) e = restore();
  if (ea) (void)hipEventDestroy(ea);
  if (eb) (void)hipEventDestroy(eb);
  cleanup();
  c->nstep = nstep0;
  c->prof = prof0;
  if (st != SW_OK) return st;
  if (e != hipSuccess) return fail(SW_EHIP, std::string("sw_autotune: ") + hipGetErrorString(e));
  if (wpb_out) *wpb_out = bw;
  if (q_out) *q_out = bq;
  return SW_OK;
}

sw_status sw_get_workgroup(const sw_ctx* c, int32_t level, int32_t kernel, int32_t* value) {
  if (!c || !value) return fail(SW_EINVAL, "NULL argument");
  for (auto& L : c->lv)
    if (L.L == level) {
      *value = kernel == 0 ? L.wpb
               : kernel == 1 ? L.face_q
                             : (L.xorder >= 0 ? L.xorder : (c->lv.size() == 1 ? 1 : 0));
      return SW_OK;
    }
  return fail(SW_EINVAL, "no such level");
}

sw_status sw_profile(sw_ctx* c, int32_t on) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  c->prof = on != 0;
  c->prof_mask = on > 1 ? (on >> 1) & 0xFF : 0xFF;
  return SW_OK;
}

sw_status sw_kernel_time(sw_ctx* c, int32_t kind, double* ms_total, int64_t* launches) {
  if (!c || !ms_total || !launches) return fail(SW_EINVAL, "NULL argument");
  if (kind < 0 || kind > 7) return fail(SW_EINVAL, "kind must be 0..7");
  for (auto& e : c->ev) {
    HIPCHK(hipEventSynchronize(e.b));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, e.a, e.b));
    c->prof_ms[e.kind] += ms;
    c->prof_n[e.kind] += e.nlaunch;
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  c->ev.clear();
  *ms_total = c->prof_ms[kind];
  *launches = c->prof_n[kind];
  return SW_OK;
}

sw_status sw_kernel_time_reset(sw_ctx* c) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  double ms;
  int64_t n;
  sw_status st = sw_kernel_time(c, 0, &ms, &n);
  if (st != SW_OK) return st;
  for (int k = 0; k < 8; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_n[k] = 0;
  }
  return SW_OK;
}

}  // extern "C"

// ---- hooks for the ensemble driver (sw_ens.hip) ----------------------------
namespace swk {
bool ctx_graph_ready(const sw_ctx* c) { return c->start_ready && c->stage_done == 0; }
int64_t ctx_steps(const sw_ctx* c) { return c->nstep; }
void ctx_set_steps(sw_ctx* c, int64_t n) { c->nstep = n; }
bool ctx_set_prof(sw_ctx* c, bool on) {
  const bool o = c->prof;
  c->prof = on;
  return o;
}
hipStream_t ctx_swap_stream(sw_ctx* c, hipStream_t s) {
  hipStream_t o = c->s;
  c->s = s;
  return o;
}
hipStream_t ctx_stream(const sw_ctx* c) { return c->s; }
int ctx_cells(const sw_ctx* c) { return c->K; }
void ctx_class(const sw_ctx* c, int* r, int* S0) {
  *r = c->r;
  *S0 = c->lv.empty() ? 0 : c->lv[0].S;
}
int api_fail(int status, const char* msg) { return (int)fail((sw_status)status, msg); }
}  // namespace swk

extern "C" {

namespace {
void fill_diag(const double* d, int64_t nstep, sw_diag* out) {
  out->min_target_mass = d[D_MINT];
  out->n_pos_viol = (int64_t)d[D_VIOL];
  out->max_newton_it = (int32_t)d[D_NEWT];
  out->n_fallback = (int64_t)d[D_FALLB];
  out->total_mass = d[D_MASS];
  out->n_r0_cells = (int64_t)d[D_NR0];
  out->nonfinite = d[D_NONF] != 0.0;
  out->dt = d[7];
  out->t = d[8];
  out->step = nstep;
}
}  // namespace

sw_status sw_diagnostics(const sw_ctx* c, sw_diag* out) {
  if (!c || !out) return fail(SW_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(c->s));
  std::vector<double> d((size_t)kMDiag * c->M);
  HIPCHK(hipMemcpy(d.data(), c->d_mdiag, d.size() * sizeof(double), hipMemcpyDeviceToHost));
  // member 0 gives dt and t; the rest is combined over the members
  double tot[kMDiag];
  for (int q = 0; q < kMDiag; ++q) tot[q] = d[q];
  for (int m = 1; m < c->M; ++m) {
    const double* e = d.data() + (size_t)m * kMDiag;
    tot[D_MINT] = std::min(tot[D_MINT], e[D_MINT]);
    tot[D_VIOL] += e[D_VIOL];
    tot[D_NEWT] = std::max(tot[D_NEWT], e[D_NEWT]);
    tot[D_FALLB] += e[D_FALLB];
    tot[D_MASS] += e[D_MASS];
    tot[D_NR0] += e[D_NR0];
    tot[D_NONF] = std::max(tot[D_NONF], e[D_NONF]);
  }
  // t and dt also before the first step (time set by sw_set_time)
  double t0 = 0.0, dt0 = 0.0;
  HIPCHK(hipMemcpy(&t0, c->d_mt, sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(&dt0, c->d_mdt, sizeof(double), hipMemcpyDeviceToHost));
  tot[7] = dt0;
  tot[8] = t0;
  fill_diag(tot, c->nstep, out);
  if (out->nonfinite) return fail(SW_ENONFINITE, "non-finite value in the state");
  return SW_OK;
}

sw_status sw_member_diagnostics(const sw_ctx* c, int32_t m, sw_diag* out) {
  if (!c || !out) return fail(SW_EINVAL, "NULL argument");
  if (m < 0 || m >= c->M) return fail(SW_EINVAL, "member index out of range");
  HIPCHK(hipStreamSynchronize(c->s));
  double d[kMDiag];
  HIPCHK(hipMemcpy(d, c->d_mdiag + (size_t)m * kMDiag, sizeof(d), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(&d[8], c->d_mt + m, sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(&d[7], c->d_mdt + m, sizeof(double), hipMemcpyDeviceToHost));
  fill_diag(d, c->nstep, out);
  if (out->nonfinite) return fail(SW_ENONFINITE, "non-finite value in the state");
  return SW_OK;
}

}  // extern "C"
